"""Calibration and closed loop on the GPU, driven through the C ABI.

Calibration (the paper's Sec. 4 requires the slope reference, the
sub-aperture indices and the reconstruction matrix before a run; the plan
measures the first two itself): push-pull interaction matrix measured with
pwfs_measure, assembled and pseudo-inverted (full SVD, nothing truncated)
on the host in FP64.

Closed loop (Sec. 3 and Tab. 2: loop control triggers sensing,
reconstruction, integration and the DM once per step; Tab. 1 "control":
integrator with a total delay of two steps):
    u(t) = c(t - delay),  r(t) = opd(t) - B u(t)   [recon_apply, alpha=-1, beta=1]
    s(t) = pwfs_measure(r(t))
    c(t) = c(t-1) + g R s(t)                        [recon_apply, alpha=g, beta=1]
All arithmetic of a step runs in the library's kernels; torch only holds
the buffers and copies them.
"""
from __future__ import annotations

import numpy as np

from ._lib import recon_apply


def interaction_matrix(plan, modes, eps_nm: float, device="cuda"):
    """IM [n_slopes, M] (FP64 host) from push-pull measurements of each mode.

    modes: host array [M, P, P]; the push/pull screens +-eps B_i are formed
    on the host (FP32) and measured in batches of the plan's batch size.
    """
    import torch
    modes = np.asarray(modes)
    M = modes.shape[0]
    ns = 2 * plan.n_valid
    IM = np.empty((ns, M))
    h = max(1, plan.batch_max // 2)
    for i0 in range(0, M, h):
        idx = list(range(i0, min(M, i0 + h)))
        blk = modes[idx].astype(np.float64) * eps_nm
        push = torch.from_numpy(np.concatenate([blk, -blk]).astype(np.float32)).to(device)
        sl = torch.empty((push.shape[0], ns), device=device)
        plan.measure_into(push, None, sl)
        sl = sl.cpu().numpy().astype(np.float64)
        n = len(idx)
        IM[:, idx] = ((sl[:n] - sl[n:]) / (2.0 * eps_nm)).T
    return IM


def pseudo_inverse(IM: np.ndarray):
    """(R, singular values): R = V diag(1/sigma) U^T, nothing truncated (FP64)."""
    U, sig, Vt = np.linalg.svd(IM, full_matrices=False)
    return (Vt.T / sig) @ U.T, sig


def calibrate(plan, modes, eps_nm: float, device="cuda"):
    """Reconstructor R [M, n_slopes] as a float32 device tensor, plus the FP64 IM and sigma."""
    import torch
    IM = interaction_matrix(plan, modes, eps_nm, device)
    R, sig = pseudo_inverse(IM)
    return torch.from_numpy(R.astype(np.float32)).to(device).contiguous(), IM, sig


class ClosedLoop:
    """Integrator loop of one sensor plan (batch 1) with a modal DM.

    With a learned reconstructor (net) the integrator input is the
    network's modal estimate from the pupil images; the linear
    reconstructor R judges it every `judge_every` steps from its own
    estimate of the modal residual, e = ||R s||, and takes over for the
    rest of the run (integrator restarted from zero) if the network output
    is not finite, if after `judge_settle` steps e has not fallen below
    half its open-loop value e(0) (the loop did not close; with large
    errors the sensor saturates, so e alone cannot show how far it
    diverged), or if e exceeds `judge_growth` times its best value since
    then (the loop is diverging)."""

    def __init__(self, plan, modes_dev, R_dev, gain: float, delay: int, net=None,
                 judge_every: int = 10, judge_growth: float = 4.0, judge_settle: int = 50):
        import torch
        self.plan, self.R, self.gain, self.delay = plan, R_dev, float(gain), int(delay)
        M, P, _ = modes_dev.shape
        self.M, self.P = M, P
        dev = modes_dev.device
        self.BKL = modes_dev.reshape(M, P * P).t().contiguous()     # [P*P, M]
        self.s = torch.empty((1, 2 * plan.n_valid), device=dev)
        self.net = net
        self.judge_every, self.judge_growth, self.judge_settle = judge_every, judge_growth, judge_settle
        self.fallback_step = None
        if net is not None:
            from .cnn import prepare
            self._prepare = prepare
            S = plan.n_sub
            self.pupils = torch.empty((1, 4, S, S), device=dev)
            self.ref = torch.empty((1, 4, S, S), device=dev)
            plan.measure_into(torch.zeros((1, P, P), device=dev), self.ref, None)
            self.valid = torch.from_numpy(plan.valid.astype(np.int32)).to(dev)
            self.x = torch.empty((1, S, S, 4), device=dev)
            self.m_lin = torch.empty((1, M), device=dev)

    def run(self, opd_seq_dev, residuals_dev=None):
        """Run len(opd_seq) steps; returns (residual OPD [T, P*P], commands c(t) [T, M])."""
        import torch
        T = opd_seq_dev.shape[0]
        P, M, d = self.P, self.M, self.delay
        dev = opd_seq_dev.device
        res = residuals_dev if residuals_dev is not None else torch.empty((T, P * P), device=dev)
        hist = torch.zeros((T + d, M), device=dev)                   # c(t) is row t + d
        learned = self.net is not None
        judged = []
        self.fallback_step = None
        for t in range(T):
            r_t = res[t:t + 1]
            r_t.copy_(opd_seq_dev[t].reshape(1, -1))
            recon_apply(self.BKL, hist[t:t + 1], -1.0, 1.0, r_t)     # u(t) = c(t - d)
            c_next = hist[t + d:t + d + 1]
            if t > 0:
                c_next.copy_(hist[t + d - 1:t + d])
            if learned:
                self.plan.measure_into(r_t.view(1, P, P), self.pupils, self.s)
                self._prepare(self.pupils, self.ref[0], self.valid, self.x)
                self.net.forward_acc(self.x, c_next, self.gain, 1.0)
                if t % self.judge_every == 0:
                    recon_apply(self.R, self.s, 1.0, 0.0, self.m_lin)
                    e = float(np.linalg.norm(self.m_lin.cpu().numpy()))
                    ok = bool(np.isfinite(c_next.cpu().numpy()).all())
                    judged.append((t, e))
                    e0 = judged[0][1]
                    settled = [v for (tt, v) in judged if tt >= self.judge_settle]
                    not_closed = t >= self.judge_settle and e > 0.5 * e0
                    diverging = len(settled) >= 2 and e > self.judge_growth * min(settled)
                    if not ok or not_closed or diverging:
                        learned = False
                        self.fallback_step = t
                        hist[: t + d + 1].zero_()
                        recon_apply(self.R, self.s, self.gain, 1.0, c_next)
            else:
                self.plan.measure_into(r_t.view(1, P, P), None, self.s)
                recon_apply(self.R, self.s, self.gain, 1.0, c_next)
        return res, hist[d:]


def residual_rms_nm(res_host: np.ndarray, pupil: np.ndarray) -> np.ndarray:
    """Piston-removed RMS over the pupil of each residual frame [T, P*P] (FP64)."""
    v = res_host.reshape(res_host.shape[0], -1)[:, pupil.ravel() > 0].astype(np.float64)
    v = v - v.mean(axis=1, keepdims=True)
    return np.sqrt((v ** 2).mean(axis=1))
