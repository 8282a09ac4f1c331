"""Literal FP64 modulated pyramid WFS: field -> focal plane -> mask -> pupil.

Test infrastructure only (see the package docstring).  Parity unpinned:
none -- every function here is pinned by tests/test_oracle_pins.py.

Paper anchors.  The pyramid object turns the pupil electric field into
pupil-plane intensity with circular modulation (Sec. 4, Tab. 1 "pyramid":
modulation radius in lambda/D, wavelength; Tab. 2 "pyr.in_ef -> out_i").
The CCD integrates that intensity into pixels (Tab. 1 "detector"), the
slope computer turns pixels into slopes using the sub-aperture indices
and a slope reference vector (Tab. 1 "slopec", Sec. 4 text on the
required calibrations).

Conventions (the paper is silent on all of them):
  * pupil: P x P circle, centre (P-1)/2, pixel inside iff r^2 <= (P/2)^2,
    optional obstruction removing r < eps P / 2; embedded at offset
    o = (N-P)/2 of the N x N grid;
  * phase phi = 2 pi opd[nm] 1e-9 / lambda;
  * modulation: theta_k = 2 pi k / K, k = 0..K-1, tilt (a_k, b_k) =
    rho (cos theta_k, sin theta_k) focal pixels with rho = r_mod N / P,
    applied as exp(i 2 pi (a_k (x - xc) + b_k (y - xc)) / N), xc = (N-1)/2;
  * focal plane: unnormalised forward FFT; pyramid mask
    M(u, v) = exp(-2 pi i Delta (|u_s| + |v_s|) / N) with u_s, v_s the
    signed frequency indices in [-N/2, N/2) (apex on bin 0); optionally
    times a circular field stop (Tab. 1 "pyramid": fov), kept where
    u_s^2 + v_s^2 <= R^2, R = (stop diameter in lambda/D) N / (2 P);
  * back to the pupil: inverse FFT with 1/N^2; intensity = mean over k;
  * pupil q = (sx > 0) + 2 (sy > 0) is the window at rows o + sy Delta,
    cols o + sx Delta (sx, sy = -1/+1), summed b x b; or, with a detector
    window S (the detector's output resolution, Tab. 1 "pyramid":
    output_resolution, pup_diam, pup_dist), resampled to S x S detector
    pixels of pitch P / S: each detector pixel integrates the
    piecewise-constant window over its footprint (a non-integer rebin);
  * valid subaperture: pupil fill fraction of its b x b block (of the
    detector pixel's footprint) >= 0.5; or the paper's pupil acquisition
    (Sec. 4 calibration script): a flat-wavefront frame taken with the
    modulation radius raised to 20 lambda/D, thresholded;
  * slopes: sx = [(I1 + I3) - (I0 + I2)] / n, sy = [(I2 + I3) - (I0 + I1)] / n,
    n = mean total flux over valid subapertures (norm_mode 0) or each
    subaperture's own total flux (norm_mode 1); ordering [sx over V; sy over V]
    with V in row-major order; reference slopes = slopes of a flat wavefront.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

_WORKERS = int(os.environ.get("ORACLE_FFT_WORKERS", "0")) or os.cpu_count() or 1


def pupil_amplitude(P: int, obstruction: float = 0.0) -> np.ndarray:
    """Binary circular pupil of diameter P pixels (float64 P x P)."""
    c = (P - 1) / 2.0
    y, x = np.mgrid[0:P, 0:P]
    r2 = (x - c) ** 2 + (y - c) ** 2
    inside = r2 <= (P / 2.0) ** 2
    if obstruction > 0.0:
        inside &= r2 >= (obstruction * P / 2.0) ** 2
    return inside.astype(np.float64)


def overlap_matrix(P: int, S: int) -> np.ndarray:
    """W [S, P]: length of [y, y + 1) inside [j P / S, (j + 1) P / S) in
    pupil pixels (exact: both ends are multiples of 1 / S)."""
    W = np.zeros((S, P))
    for j in range(S):
        for y in range(P):
            ov = min((y + 1) * S, (j + 1) * P) - max(y * S, j * P)
            if ov > 0:
                W[j, y] = ov / S
    return W


def rebin(win: np.ndarray, S: int) -> np.ndarray:
    """Detector pixels [S, S] of a P x P window: the integral of the
    piecewise-constant image over each pixel's footprint (pupil-pixel area
    units), out[j, i] = sum_y,x W[j, y] W[i, x] win[y, x]."""
    W = overlap_matrix(win.shape[0], S)
    return W @ win @ W.T


def valid_subapertures(A: np.ndarray, b: int, det_window: int = 0) -> np.ndarray:
    """Indices j = iy * S + ix (ascending) of subapertures whose b x b block
    of the pupil (detector pixel footprint with a detector window) is at
    least half filled."""
    P = A.shape[0]
    if det_window:
        S = det_window
        fill = rebin(A, S) / (P / S) ** 2
    else:
        S = P // b
        fill = A.reshape(S, b, S, b).mean(axis=(1, 3))
    return np.flatnonzero(fill.ravel() >= 0.5).astype(np.int64)


def acquire_valid(pupils: np.ndarray, thr: float) -> np.ndarray:
    """Pupil acquisition on a detector frame [4, S, S] (the paper's
    calibration thresholds a flat-wavefront frame taken with a large
    modulation radius; its thresholds are not given): subapertures where the
    sum of the four pupil images reaches thr times its maximum."""
    tot = pupils.sum(axis=0).ravel()
    return np.flatnonzero(tot >= thr * tot.max()).astype(np.int64)


def modulation_offsets(cfg) -> tuple[np.ndarray, np.ndarray]:
    """Tilt (a_k, b_k) in focal-plane pixels for the K modulation points."""
    K = cfg.n_mod
    rho = cfg.mod_radius_lod * cfg.n_fft / cfg.n_pupil
    th = 2.0 * np.pi * np.arange(K) / K
    return rho * np.cos(th), rho * np.sin(th)


def pyramid_mask(N: int, delta: int) -> np.ndarray:
    """Four-face pyramid phase mask on the unshifted FFT grid (N x N complex)."""
    us = np.abs(np.fft.fftfreq(N, 1.0 / N))          # |signed index|, exact ints
    return np.exp(-2j * np.pi * delta * (us[None, :] + us[:, None]) / N)


def field_stop_mask(N: int, P: int, diameter_lod: float) -> np.ndarray:
    """Circular focal-plane stop of the given diameter (lambda/D units of the
    modulation radius) on the unshifted N x N grid (float64 0/1)."""
    us = np.fft.fftfreq(N, 1.0 / N)
    R = 0.5 * diameter_lod * N / P
    return ((us[None, :] ** 2 + us[:, None] ** 2) <= R * R).astype(np.float64)


def sensor_mask(cfg) -> np.ndarray:
    """Pyramid mask, times the field stop when the configuration has one."""
    M = pyramid_mask(cfg.n_fft, cfg.delta)
    fs = getattr(cfg, "field_stop_lod", 0.0)
    return M * field_stop_mask(cfg.n_fft, cfg.n_pupil, fs) if fs > 0 else M


def _field(cfg, opd_nm: np.ndarray, A: np.ndarray) -> np.ndarray:
    N, P = cfg.n_fft, cfg.n_pupil
    o = (N - P) // 2
    phi = 2.0 * np.pi * np.asarray(opd_nm, np.float64) * 1e-9 / cfg.wavelength_m
    E = np.zeros((N, N), np.complex128)
    E[o:o + P, o:o + P] = A * np.exp(1j * phi)
    return E


def intensity(cfg, opd_nm: np.ndarray, A: np.ndarray | None = None,
              mask: np.ndarray | None = None, offsets=None) -> np.ndarray:
    """Modulated pupil-plane intensity I (N x N float64), mean over k.

    opd_nm is the P x P optical path difference (y rows, x columns).
    mask / offsets override the pyramid mask and the modulation tilts.
    """
    N = cfg.n_fft
    if A is None:
        A = pupil_amplitude(cfg.n_pupil, cfg.obstruction)
    if mask is None:
        mask = sensor_mask(cfg)
    a, b = modulation_offsets(cfg) if offsets is None else offsets
    E = _field(cfg, opd_nm, A)
    g = np.arange(N) - (N - 1) / 2.0
    I = np.zeros((N, N))
    for ak, bk in zip(a, b):
        ramp = np.exp(2j * np.pi * (ak * g[None, :] + bk * g[:, None]) / N)
        focal = sfft.fft2(E * ramp, workers=_WORKERS)
        back = sfft.ifft2(mask * focal, workers=_WORKERS)
        I += back.real ** 2 + back.imag ** 2
    return I / len(a)


def pupil_images(cfg, I: np.ndarray) -> np.ndarray:
    """Four binned pupil images [4, S, S] cut from the N x N intensity."""
    N, P, b = cfg.n_fft, cfg.n_pupil, cfg.n_bin
    dw = getattr(cfg, "det_window", 0)
    S = dw if dw else P // b
    o = (N - P) // 2
    d = cfg.delta
    out = np.empty((4, S, S))
    for q in range(4):
        sx = 1 if q & 1 else -1
        sy = 1 if q & 2 else -1
        r0, c0 = o + sy * d, o + sx * d
        win = I[r0:r0 + P, c0:c0 + P]
        out[q] = rebin(win, S) if dw else win.reshape(S, b, S, b).sum(axis=(1, 3))
    return out


def slopes(pupils: np.ndarray, valid: np.ndarray, norm_mode: int = 0) -> np.ndarray:
    """Normalised x/y slopes [sx over V ; sy over V] from [4, S, S] pupils."""
    I = pupils.reshape(4, -1)[:, valid]
    total = I.sum(axis=0)
    n = total.mean() if norm_mode == 0 else total
    sx = ((I[1] + I[3]) - (I[0] + I[2])) / n
    sy = ((I[2] + I[3]) - (I[0] + I[1])) / n
    return np.concatenate([sx, sy])


class Oracle:
    """One sensor: pupil, valid list and reference slopes fixed at construction."""

    def __init__(self, cfg, A: np.ndarray | None = None, valid: np.ndarray | None = None):
        self.cfg = cfg
        self.A = pupil_amplitude(cfg.n_pupil, cfg.obstruction) if A is None else np.asarray(A, np.float64)
        self.valid = (valid_subapertures(self.A, cfg.n_bin, getattr(cfg, "det_window", 0)) if valid is None
                      else np.asarray(valid, np.int64))
        flat = np.zeros((cfg.n_pupil, cfg.n_pupil))
        self.ref_pupils = pupil_images(cfg, intensity(cfg, flat, self.A))
        self.s_ref = slopes(self.ref_pupils, self.valid, cfg.norm_mode)

    @property
    def n_valid(self) -> int:
        return int(self.valid.size)

    def pupils(self, opd_nm: np.ndarray) -> np.ndarray:
        return pupil_images(self.cfg, intensity(self.cfg, opd_nm, self.A))

    def measure(self, opd_nm: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
        """(pupils [4,S,S], reference-subtracted slopes [2 n_valid])."""
        p = self.pupils(opd_nm)
        return p, slopes(p, self.valid, self.cfg.norm_mode) - self.s_ref

    def measure_batch(self, opd_nm: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
        res = [self.measure(o) for o in np.asarray(opd_nm)]
        return np.stack([r[0] for r in res]), np.stack([r[1] for r in res])
