"""FP64 modal reconstructor, calibration and integrator loop.

Test infrastructure only (see the package docstring).

Paper anchors: the slope computer feeds a modal reconstructor whose
reconstruction matrix must be calibrated before the run (Sec. 4 text;
Tab. 1 "modalrec"), followed by an integrator controller with a gain per
mode and a total delay in steps (Tab. 1 "control": type INT, delay 2);
the loop runs sense -> reconstruct -> integrate -> DM once per step
(Sec. 3, Tab. 2 "loop.add" order).

Conventions: the interaction matrix is measured push-pull with amplitude
eps nm on each mode, IM[:, i] = (s(+eps B_i) - s(-eps B_i)) / (2 eps);
the reconstructor is the Moore-Penrose inverse from a full SVD with no
singular value dropped; the integrator is c(t) = c(t-1) + g R s(t) and
the DM applies u(t) = c(t - d) with c(t) = 0 for t < 0.
"""
from __future__ import annotations

import numpy as np


def interaction_matrix(measure, modes_nm: np.ndarray, eps_nm: float) -> np.ndarray:
    """IM [n_slopes, M] from a slope function measure(opd) -> slopes."""
    cols = []
    for B in modes_nm:
        cols.append((measure(eps_nm * B) - measure(-eps_nm * B)) / (2.0 * eps_nm))
    return np.stack(cols, axis=1)


def pseudo_inverse(IM: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """(R = V diag(1/sigma) U^T, sigma) from the thin SVD of IM, nothing truncated."""
    U, sig, Vt = np.linalg.svd(IM, full_matrices=False)
    return (Vt.T / sig) @ U.T, sig


def residual_rms_nm(res: np.ndarray, A: np.ndarray) -> float:
    """Piston-removed RMS of one residual OPD over the pupil pixels."""
    v = res[A > 0]
    return float(np.sqrt(np.mean((v - v.mean()) ** 2)))


def closed_loop(measure, opd_seq_nm: np.ndarray, modes_nm: np.ndarray, R: np.ndarray,
                gain: float, delay: int, A: np.ndarray):
    """Run the integrator loop; returns (per-step residual RMS [T], commands [T, M]).

    At step t: u(t) = c(t - delay); r(t) = opd(t) - sum_i u_i(t) B_i;
    s(t) = measure(r(t)); c(t) = c(t-1) + gain R s(t).
    """
    T = len(opd_seq_nm)
    M = modes_nm.shape[0]
    flat_modes = modes_nm.reshape(M, -1)
    c_hist = np.zeros((T, M))
    rms = np.zeros(T)
    c = np.zeros(M)
    for t in range(T):
        u = c_hist[t - delay] if t - delay >= 0 else np.zeros(M)
        r = np.asarray(opd_seq_nm[t], np.float64) - (u @ flat_modes).reshape(opd_seq_nm[t].shape)
        rms[t] = residual_rms_nm(r, A)
        c = c + gain * (R @ measure(r))
        c_hist[t] = c
    return rms, c_hist


def loop_residual_nm(rms: np.ndarray, settle: int) -> float:
    """sqrt of the mean square residual over steps t >= settle."""
    return float(np.sqrt(np.mean(rms[settle:] ** 2)))
