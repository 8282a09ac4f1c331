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


def acquire_valid(cfg, pupil_amp=None, thr: float = 0.5, mod_radius_lod: float = 20.0, n_mod: int = 128,
                  device="cuda") -> np.ndarray:
    """Pupil acquisition (the paper's Sec. 4 calibration script): a flat
    wavefront measured through the library with the modulation radius raised
    (20 lambda/D), then thresholded on the host: the subapertures where the
    sum of the four pupil images reaches thr times its maximum (the paper's
    thresholds are not given; one relative threshold is used).  Returns the
    ascending index list for Plan.set_valid."""
    import dataclasses
    import torch
    from ._lib import Plan
    acq = Plan(dataclasses.replace(cfg, mod_radius_lod=float(mod_radius_lod), n_mod=int(n_mod)), batch_max=1,
               pupil_amp=pupil_amp)
    try:
        P = cfg.n_pupil
        pupils, _ = acq.measure(torch.zeros((1, P, P), dtype=torch.float32, device=device))
        tot = pupils[0].double().sum(dim=0).cpu().numpy().ravel()
    finally:
        acq.close()
    return np.flatnonzero(tot >= thr * tot.max()).astype(np.int32)


class ClosedLoop:
    """Integrator loop of one sensor plan (batch 1) with a modal DM.

    With a learned reconstructor (net) the integrator input is the linear
    estimate plus the network's correction from the pupil images,
    c(t) = c(t-1) + g (R s(t) + f(x(t))).  The linear reconstructor judges
    it every `judge_every` steps by measuring the sensor's optical gain at
    the current residual r(t): push-pull probes r(t) +- a B_k of a few modes
    (a = probe_nm), measured and reconstructed by R, give
    gamma = mean_k [R (s+ - s-)]_k / (2 a), the quantity a modal dither
    measures on a real system.  gamma is ~1 at a flat wavefront, drops as
    the residual grows and goes to ~0 once the sensor has lost track (neither
    the slope RMS nor the size of R s shows this: both shrink again at very
    large residuals, where the phase wraps inside each subaperture).  The
    linear reconstructor takes over for the rest of the run (integrator
    restarted from zero) if the commands are not finite, if after
    `judge_settle` steps gamma is below `gain_min` (the loop did not close),
    or if gamma falls below `gain_drop` times its best value since then (the
    loop is diverging).  `judged` keeps the (t, gamma) pairs of the last
    run.  The 2 x (number of probe modes) probe frames are measured as one
    batch by a second plan of the same geometry (noiseless, the loop plan's
    valid list); the reference slopes cancel in s+ - s-."""

    def __init__(self, plan, modes_dev, R_dev, gain: float, delay: int, net=None,
                 judge_every: int = 10, judge_settle: int = 50, gain_min: float = 0.1,
                 gain_drop: float = 0.5, probe_modes=(0, 1, 20, 100), probe_nm: float = 20.0):
        import torch
        self.plan, self.R, self.gain, self.delay = plan, R_dev, float(gain), int(delay)
        M, P, _ = modes_dev.shape
        self.M, self.P = M, P
        dev = modes_dev.device
        self.BKL = modes_dev.reshape(M, P * P).t().contiguous()     # [P*P, M]
        self.s = torch.empty((1, 2 * plan.n_valid), device=dev)
        self.net = net
        self.judge_every, self.judge_settle = judge_every, judge_settle
        self.gain_min, self.gain_drop = gain_min, gain_drop
        self.fallback_step = None
        self.judged = []
        if net is not None:
            from .cnn import prepare
            self._prepare = prepare
            S = plan.n_sub
            self.pupils = torch.empty((1, 4, S, S), device=dev)
            self.ref = torch.empty((1, 4, S, S), device=dev)
            plan.measure_into(torch.zeros((1, P, P), device=dev), self.ref, None)
            self.valid = torch.from_numpy(plan.valid.astype(np.int32)).to(dev)
            self.x = torch.empty((1, S, S, 4), device=dev)
            self.probe_modes = [int(k) for k in probe_modes if 0 <= int(k) < M]
            self.probe_nm = float(probe_nm)
            npb = len(self.probe_modes)
            coef = np.zeros((2 * npb, M), np.float32)
            for j, k in enumerate(self.probe_modes):
                coef[2 * j, k], coef[2 * j + 1, k] = self.probe_nm, -self.probe_nm
            self.probe_coef = torch.from_numpy(coef).to(dev)
            from ._lib import Plan
            self.probe_plan = Plan(plan.cfg, batch_max=2 * npb, pupil_amp=plan.pupil)
            if not np.array_equal(self.probe_plan.valid, plan.valid):
                self.probe_plan.set_valid(plan.valid)
            self.probe_screen = torch.empty((2 * npb, P * P), device=dev)
            self.probe_s = torch.empty((2 * npb, 2 * plan.n_valid), device=dev)
            self.probe_est = torch.empty((2 * npb, M), device=dev)

    def _probe(self, r_t) -> None:
        """Launch the push-pull probes around the residual r_t [1, P*P] and
        their reconstruction into probe_est (library kernels)."""
        P = self.P
        n = self.probe_screen.shape[0]
        self.probe_screen.copy_(r_t.expand(n, -1))
        recon_apply(self.BKL, self.probe_coef, 1.0, 1.0, self.probe_screen)    # r_t +- a B_k, all probes at once
        self.probe_plan.measure_into(self.probe_screen.view(n, P, P), None, self.probe_s)
        recon_apply(self.R, self.probe_s, 1.0, 0.0, self.probe_est)

    def _gain_of(self, est: np.ndarray) -> float:
        est = est.astype(np.float64)
        g = [(est[2 * j, k] - est[2 * j + 1, k]) / (2.0 * self.probe_nm) for j, k in enumerate(self.probe_modes)]
        return float(np.mean(g))

    def optical_gain(self, r_t) -> float:
        """Mean push-pull response of the linear reconstructor to the probe
        modes around the residual r_t [1, P*P] (library kernels; host mean)."""
        self._probe(r_t)
        return self._gain_of(self.probe_est.cpu().numpy())

    def _judge(self, t: int, r_t, c_next) -> bool:
        """True when the learned reconstructor must hand over (host logic).
        The probes are launched before the commands are read back, so one
        transfer (one wait for the device) serves both."""
        import torch
        self._probe(r_t)
        both = torch.cat([c_next.reshape(-1), self.probe_est.reshape(-1)]).cpu().numpy()
        ok = bool(np.isfinite(both[:c_next.numel()]).all())
        if not ok:
            self.judged.append((t, float("nan")))
            return True
        gam = self._gain_of(both[c_next.numel():].reshape(self.probe_est.shape))
        self.judged.append((t, gam))
        if t < self.judge_settle:
            return False
        settled = [v for (tt, v) in self.judged if tt >= self.judge_settle]
        return gam < self.gain_min or gam < self.gain_drop * max(settled)

    def run(self, opd_seq_dev, residuals_dev=None, state=None):
        """Run len(opd_seq) steps; returns (residual OPD [T, P*P], commands c(t) [T, M]).

        Without state the loop starts at t = 0 from zero commands.  With the
        state of an earlier run (its `state` attribute, or load_state) it
        continues that run: the delay line c(t0 - d) ... c(t0 - 1), the
        reconstructor in use (learned, or linear after a hand-over), the
        judge's record and the step count t0 (which sets the judge's
        schedule) are restored, so running T1 steps and then T2 from the
        state equals one run of T1 + T2 steps bit for bit.  After the run,
        `state` holds the loop's state at its end.  At a hand-over at step t
        the integrator restarts from zero: c(t - d + 1) ... c(t - 1), still
        in the delay line, are set to zero (so they read zero in the returned
        commands) and c(t) = g R s(t)."""
        import torch
        T = opd_seq_dev.shape[0]
        P, M, d = self.P, self.M, self.delay
        dev = opd_seq_dev.device
        res = residuals_dev if residuals_dev is not None else torch.empty((T, P * P), device=dev)
        hist = torch.zeros((T + d, M), device=dev)                   # c(t0 + t) is row t + d
        learned = self.net is not None
        t0 = 0
        if state is None:
            self.judged = []
            self.fallback_step = None
        else:
            if d < 1:
                raise ValueError("resuming needs delay >= 1")
            cmd = torch.as_tensor(state["commands"], dtype=torch.float32)
            if tuple(cmd.shape) != (d, M):
                raise ValueError(f"state holds commands of shape {tuple(cmd.shape)}, the loop needs ({d}, {M})")
            if state["learned"] and self.net is None:
                raise ValueError("state of a learned loop: the loop needs the network")
            hist[:d].copy_(cmd.to(dev))
            learned = learned and bool(state["learned"])
            t0 = int(state["t"])
            self.judged = [tuple(v) for v in state["judged"]]
            self.fallback_step = None if state["fallback_step"] < 0 else int(state["fallback_step"])
        for t in range(T):
            ta = t0 + t
            r_t = res[t:t + 1]
            r_t.copy_(opd_seq_dev[t].reshape(1, -1))
            recon_apply(self.BKL, hist[t:t + 1], -1.0, 1.0, r_t)     # u(t) = c(t - d)
            c_next = hist[t + d:t + d + 1]
            if ta > 0:
                c_next.copy_(hist[t + d - 1:t + d])
            if learned:
                self.plan.measure_into(r_t.view(1, P, P), self.pupils, self.s)
                recon_apply(self.R, self.s, self.gain, 1.0, c_next)
                self._prepare(self.pupils, self.ref[0], self.valid, self.x)
                self.net.forward_acc(self.x, c_next, self.gain, 1.0)
                if ta % self.judge_every == 0 and self._judge(ta, r_t, c_next):
                    learned = False
                    self.fallback_step = ta
                    hist[t + 1:t + d + 1].zero_()                    # the delay line still to be read
                    recon_apply(self.R, self.s, self.gain, 1.0, c_next)
            else:
                self.plan.measure_into(r_t.view(1, P, P), None, self.s)
                recon_apply(self.R, self.s, self.gain, 1.0, c_next)
        self.state = {"t": t0 + T, "commands": hist[T:T + d].clone(), "learned": learned,
                      "fallback_step": -1 if self.fallback_step is None else self.fallback_step,
                      "judged": list(self.judged)}
        return res, hist[d:]

    def run_graph(self, opd_seq_dev, residuals_dev=None, steps_per_graph: int = 50):
        """run() (from t = 0) replayed from captured HIP graphs
        (torch.cuda.CUDAGraph) of up to `steps_per_graph` steps each: the
        same library calls in the same order on static buffers, so the same
        results bit for bit.  A graph advances a window of n steps: the
        window's inputs are copied in once, its residuals and commands out
        once, and the delay line is the command window itself (hist_ext[j] =
        c(t - d) for step t = t0 + j, rows 0..d-1 carried over from the
        previous window).  With the learned reconstructor a window ends at
        each of the judge's steps (t a multiple of judge_every, t = 0 first)
        and the judge runs between replays as in run(), its probes launched
        one by one; after a hand-over the linear reconstructor's windows
        follow.  One graph is captured per (reconstructor, window length),
        kept on the loop object for later runs with the same steps_per_graph.
        Afterwards `state` holds the loop's state as after run().  Needs
        delay >= 1 and a noiseless sensor (a detector's frame counter would
        be frozen into the graph)."""
        import torch
        if self.delay < 1:
            raise ValueError("graph replay needs delay >= 1")
        det = getattr(self.plan, "detector", None)
        if det is not None and det()["gain"] > 0.0:
            raise ValueError("graph replay needs a noiseless sensor")
        T = opd_seq_dev.shape[0]
        P, M, d = self.P, self.M, self.delay
        dev = opd_seq_dev.device
        res = residuals_dev if residuals_dev is not None else torch.empty((T, P * P), device=dev)
        hist = torch.empty((T, M), device=dev)
        L = max(1, min(int(steps_per_graph), T))
        cache = getattr(self, "_graphs", None)
        if cache is None or cache["L"] != L or cache["device"] != dev:
            cache = {"L": L, "device": dev, "graphs": {},
                     "bufs": (torch.zeros((L, P * P), device=dev), torch.zeros((L, P * P), device=dev),
                              torch.zeros((L + d, M), device=dev))}
            self._graphs = cache
        opd_win, res_win, hist_ext = cache["bufs"]

        def window(n, learned):
            for j in range(n):
                r = res_win[j:j + 1]
                r.copy_(opd_win[j:j + 1])
                recon_apply(self.BKL, hist_ext[j:j + 1], -1.0, 1.0, r)          # u(t) = c(t - d)
                c = hist_ext[j + d:j + d + 1]
                c.copy_(hist_ext[j + d - 1:j + d])                              # c(t - 1)
                if learned:
                    self.plan.measure_into(r.view(1, P, P), self.pupils, self.s)
                    recon_apply(self.R, self.s, self.gain, 1.0, c)
                    self._prepare(self.pupils, self.ref[0], self.valid, self.x)
                    self.net.forward_acc(self.x, c, self.gain, 1.0)            # c(t) = c(t-1) + g (R s + f(x))
                else:
                    self.plan.measure_into(r.view(1, P, P), None, self.s)
                    recon_apply(self.R, self.s, self.gain, 1.0, c)              # c(t) = c(t-1) + g R s(t)

        def graph(n, learned):
            key = (learned, n)
            if key not in cache["graphs"]:
                carry = hist_ext[:d].clone()                                   # the warm-up overwrites the window
                side = torch.cuda.Stream(device=dev)
                side.wait_stream(torch.cuda.current_stream(dev))
                with torch.cuda.stream(side):
                    window(n, learned)                                         # warm-up outside the capture
                torch.cuda.current_stream(dev).wait_stream(side)
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g):
                    window(n, learned)
                hist_ext[:d].copy_(carry)
                cache["graphs"][key] = g
            return cache["graphs"][key]

        learned = self.net is not None
        self.judged = []
        self.fallback_step = None
        je = self.judge_every
        if not learned:
            for n in {L, T % L} - {0}:
                graph(n, False)
        hist_ext.zero_()
        t0 = 0
        while t0 < T:
            if learned:
                judge_t = -(-t0 // je) * je                                    # first judge step >= t0
                n = min(judge_t - t0 + 1, T - t0, L)
            else:
                n = min(L, T - t0)
            g = graph(n, learned)
            opd_win[:n].copy_(opd_seq_dev[t0:t0 + n].reshape(n, -1))
            g.replay()
            ta = t0 + n - 1
            if learned and ta % je == 0 and self._judge(ta, res_win[n - 1:n], hist_ext[n - 1 + d:n + d]):
                learned = False
                self.fallback_step = ta
                hist_ext[n:n + d].zero_()                                      # the delay line still to be read
                recon_apply(self.R, self.s, self.gain, 1.0, hist_ext[n - 1 + d:n + d])
            res[t0:t0 + n].copy_(res_win[:n])
            hist[t0:t0 + n].copy_(hist_ext[d:d + n])
            hist_ext[:d].copy_(hist_ext[n:n + d].clone())
            t0 += n
        self.state = {"t": T, "commands": hist_ext[:d].clone(), "learned": learned,
                      "fallback_step": -1 if self.fallback_step is None else self.fallback_step,
                      "judged": list(self.judged)}
        return res, hist


class BatchedLoop:
    """B independent integrator loops (Monte-Carlo realisations: different
    screens, same sensor, reconstructor and controller) advanced together,
    so each step is one pwfs_measure of B frames, one recon_apply over B
    slope vectors and one batched DM product:
        u_b(t) = c_b(t - delay),  r_b(t) = opd_b(t) - B u_b(t)
        c_b(t) = c_b(t-1) + g R s(r_b(t))
    Each realisation follows exactly the equations of ClosedLoop; only the
    batching (and with it the plan's work split, i.e. the FP32 summation
    order of the modulation sum) differs.  B <= plan.batch_max."""

    def __init__(self, plan, modes_dev, R_dev, gain: float, delay: int):
        import torch
        self.plan, self.R, self.gain, self.delay = plan, R_dev, float(gain), int(delay)
        M, P, _ = modes_dev.shape
        self.M, self.P = M, P
        self.BKL = modes_dev.reshape(M, P * P).t().contiguous()     # [P*P, M]

    def run(self, opd_seq_dev, residuals_dev=None):
        """opd_seq_dev [T, B, P, P]; returns (residual OPD [T, B, P*P], commands [T, B, M])."""
        import torch
        T, B = opd_seq_dev.shape[0], opd_seq_dev.shape[1]
        if B > self.plan.batch_max:
            raise ValueError(f"{B} realisations exceed the plan's batch_max {self.plan.batch_max}")
        P, M, d = self.P, self.M, self.delay
        dev = opd_seq_dev.device
        res = residuals_dev if residuals_dev is not None else torch.empty((T, B, P * P), device=dev)
        hist = torch.zeros((T + d, B, M), device=dev)                # c(t) is row t + d
        s = torch.empty((B, 2 * self.plan.n_valid), device=dev)
        for t in range(T):
            r_t = res[t]
            r_t.copy_(opd_seq_dev[t].reshape(B, -1))
            recon_apply(self.BKL, hist[t], -1.0, 1.0, r_t)
            c_next = hist[t + d]
            if t > 0:
                c_next.copy_(hist[t + d - 1])
            self.plan.measure_into(r_t.view(B, P, P), None, s)
            recon_apply(self.R, s, self.gain, 1.0, c_next)
        return res, hist[d:]


def residual_rms_nm(res_host: np.ndarray, pupil: np.ndarray) -> np.ndarray:
    """Piston-removed RMS over the pupil of each residual frame [T, P*P] (FP64)."""
    v = res_host.reshape(res_host.shape[0], -1)[:, pupil.ravel() > 0].astype(np.float64)
    v = v - v.mean(axis=1, keepdims=True)
    return np.sqrt((v ** 2).mean(axis=1))


def save_state(path: str, state: dict, meta: dict | None = None) -> None:
    """Write a ClosedLoop state (plus free-form metadata such as the screen
    seed and the frozen-flow offset, kept as JSON) to an .npz of plain arrays."""
    import json
    cmd = state["commands"]
    cmd = cmd.detach().cpu().numpy() if hasattr(cmd, "detach") else np.asarray(cmd)
    judged = np.asarray(state["judged"], np.float64).reshape(-1, 2)
    np.savez(path, t=np.int64(state["t"]), commands=np.asarray(cmd, np.float32),
             learned=np.bool_(state["learned"]), fallback_step=np.int64(state["fallback_step"]),
             judged=judged, meta=np.array(json.dumps(meta or {}, sort_keys=True)))


def load_state(path: str):
    """(state, meta) from save_state's file (read without unpickling)."""
    import json
    with np.load(path, allow_pickle=False) as z:
        state = {"t": int(z["t"]), "commands": z["commands"].copy(), "learned": bool(z["learned"]),
                 "fallback_step": int(z["fallback_step"]),
                 "judged": [(int(a), float(b)) for a, b in z["judged"]]}
        return state, json.loads(str(z["meta"]))
