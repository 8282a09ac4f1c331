"""Learned modal reconstructor: training-set generation on the GPU, training
loop and checkpoints, driven through the C ABI (pwfs_measure, recon_apply,
pwfs_cnn_*).

The learned reconstructor estimates the modal coefficients as the linear
estimate plus a network correction, c = R s + f(x): the network sees the
pupil images (pwfs_cnn_prepare) and learns what the linear reconstructor
misses, chiefly the loss of pyramid sensitivity (optical gain) when the
residual is large and the non-linear response to strong aberrations; a
network that outputs zero is the linear reconstructor.

Training inputs are simulator frames: seeded screens (open loop) and
partially corrected screens (residuals of linear closed loops, or screens
with a random fraction of their first KL modes removed through the DM
path), measured by the pyramid plan.  Labels are the KL coefficients of the
measured screen minus the linear estimate, c_true - R s (both products
through recon_apply), divided by one global scale.  After training the
scale is folded into the last layer, so the network outputs nm, the same
units as R s.
"""
from __future__ import annotations

import numpy as np

from ._lib import recon_apply
from .cnn import CNN, prepare, he_init, PARAM_ORDER


class TrainingSet:
    """x [F, S, S, 4] network inputs, y [F, M] scaled labels (device),
    frame_rms [F] RMS over the modes of each frame's true coefficients, nm
    (host), w [F] per-frame loss weights or None."""

    def __init__(self, x, y, label_scale, frame_rms, w=None):
        self.x, self.y, self.label_scale, self.frame_rms, self.w = x, y, label_scale, frame_rms, w

    def set_relative_weights(self, floor_nm: float):
        """Per-frame loss weights 1 / (frame_rms^2 + floor^2), normalised to
        mean 1: each frame's error counts relative to the size of its
        wavefront error, so the small residuals of a closed loop are learned
        as accurately as large open-loop aberrations."""
        import torch
        w = 1.0 / (self.frame_rms.astype(np.float64) ** 2 + float(floor_nm) ** 2)
        w /= w.mean()
        self.w = torch.from_numpy(w.astype(np.float32)).to(self.y.device)


def projector(modes: np.ndarray, pupil: np.ndarray, device="cuda"):
    """Projection matrix [M, P*P] (modes / n_pix) as a device tensor: c = Proj opd."""
    import torch
    n_pix = float((pupil > 0).sum())
    M = modes.shape[0]
    return torch.from_numpy((modes.reshape(M, -1) / n_pix).astype(np.float32)).to(device).contiguous()


class ResidualBank:
    """Residual screens of linear closed loops (frozen flow, random r0),
    the 'partially corrected phase' half of the training set.  Frames are
    drawn with one of the 8 square symmetries (a symmetry of a screen is a
    screen; its label is recomputed from the transformed screen)."""

    def __init__(self, frames_dev):
        self.frames = frames_dev            # [F, P, P] float32, device

    @staticmethod
    def from_loops(plan1, modes_dev, R_dev, cfg, L0_m, wind_m_s, rate_hz, n_loops, steps, settle, seed,
                   r0_range, gain, delay, stride=1):
        import torch
        from synth.configs import AtmoConfig
        from synth.screens import frozen_flow_sequence
        from .loop import ClosedLoop
        rng = np.random.default_rng(seed)
        P = cfg.n_pupil
        out = []
        for i in range(n_loops):
            r0 = float(rng.uniform(*r0_range))
            atm = AtmoConfig(r0_m=r0, L0_m=L0_m, wind_m_s=wind_m_s, frame_rate_hz=rate_hz)
            seq = torch.from_numpy(frozen_flow_sequence(cfg, atm, steps, seed=int(rng.integers(1 << 30)),
                                                        screen_n=2048)).to(modes_dev.device)
            res, _ = ClosedLoop(plan1, modes_dev, R_dev, gain, delay).run(seq)
            out.append(res[settle::stride].reshape(-1, P, P).clone())
        return ResidualBank(torch.cat(out))

    def draw(self, rng: np.random.Generator, n: int):
        import torch
        idx = torch.from_numpy(rng.integers(0, self.frames.shape[0], size=n)).to(self.frames.device)
        x = self.frames.index_select(0, idx)
        sym = int(rng.integers(8))
        if sym & 1:
            x = x.flip(1)
        if sym & 2:
            x = x.flip(2)
        if sym & 4:
            x = x.transpose(1, 2)
        return x.contiguous()


def make_training_set(plan, bank, R_dev, modes: np.ndarray, pupil: np.ndarray, n_frames: int, seed: int,
                      r0_range=(0.06, 0.2), corrected_fraction=0.5, batch=256, label_scale=None,
                      residuals: "ResidualBank | None" = None, device="cuda") -> TrainingSet:
    """Generate n_frames (input, label) pairs on the GPU.  A fraction
    corrected_fraction of each batch is partially corrected: residual
    screens of linear closed loops when a ResidualBank is given, otherwise
    open-loop screens with a random fraction of their first KL modes
    removed through the DM path.  Labels: (c_true - R s) / label_scale."""
    import torch
    rng = np.random.default_rng(seed)
    P, S, M = plan.cfg.n_pupil, plan.n_sub, modes.shape[0]
    ns = 2 * plan.n_valid
    proj = projector(modes, pupil, device)
    BKL = torch.from_numpy(modes.reshape(M, -1).T.astype(np.float32)).to(device).contiguous()
    valid = torch.from_numpy(plan.valid.astype(np.int32)).to(device)
    zero = torch.zeros((1, P, P), device=device)
    ref = torch.empty((1, 4, S, S), device=device)
    plan.measure_into(zero, ref, None)
    X = torch.empty((n_frames, S, S, 4), device=device)
    Y = torch.empty((n_frames, M), device=device)
    rms = np.empty(n_frames)
    pup = torch.empty((plan.batch_max, 4, S, S), device=device)
    sl = torch.empty((batch, ns), device=device)
    ct = torch.empty((batch, M), device=device)
    for i0 in range(0, n_frames, batch):
        n = min(batch, n_frames - i0)
        opd_h, _ = bank.draw(rng, n, r0_range)
        opd = torch.from_numpy(opd_h).to(device).reshape(n, P * P).contiguous()
        # Partial correction of a random subset of frames: remove alpha * c_i B_i for
        # i < n_corr (coefficients scaled on the host, DM path through recon_apply).
        n_cor = int(round(corrected_fraction * n))
        if n_cor and residuals is not None:
            opd[:n_cor] = residuals.draw(rng, n_cor).reshape(n_cor, P * P)
        elif n_cor:
            c = recon_apply(proj, opd[:n_cor]).cpu().numpy()                 # [n_cor, M]
            for j in range(n_cor):
                c[j, rng.integers(20, M + 1):] = 0.0
                c[j] *= rng.uniform(0.5, 1.0)
            recon_apply(BKL, torch.from_numpy(c).to(device), -1.0, 1.0, opd[:n_cor])
        for b0 in range(0, n, plan.batch_max):
            nb = min(plan.batch_max, n - b0)
            plan.measure_into(opd[b0:b0 + nb].view(nb, P, P), pup[:nb], sl[b0:b0 + nb])
            prepare(pup[:nb], ref[0], valid, X[i0 + b0:i0 + b0 + nb])
        recon_apply(proj, opd, 1.0, 0.0, ct[:n])
        c_h = ct[:n].cpu().numpy().astype(np.float64)
        rms[i0:i0 + n] = np.sqrt(np.mean(c_h * c_h, axis=1))
        if label_scale is None:
            lin = recon_apply(R_dev, sl[:n]).cpu().numpy().astype(np.float64)
            label_scale = float(np.sqrt(np.mean((c_h - lin) ** 2)))
        y = Y[i0:i0 + n]
        recon_apply(proj, opd, 1.0 / label_scale, 0.0, y)
        recon_apply(R_dev, sl[:n], -1.0 / label_scale, 1.0, y)
    return TrainingSet(X, Y, label_scale, rms)


def train(net: CNN, data: TrainingSet, epochs: int, batch: int, lr: float, seed: int, log=None):
    """Adam over shuffled mini-batches; returns the mean loss of each epoch."""
    import torch
    n = data.x.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    loss = torch.empty(1, device=data.x.device)
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(data.x.device)
        acc, steps = 0.0, 0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            xb = data.x.index_select(0, idx).contiguous()
            yb = data.y.index_select(0, idx).contiguous()
            wb = data.w.index_select(0, idx).contiguous() if data.w is not None else None
            net.train_step(xb, yb, lr, loss=loss, weights=wb)
            if steps % 16 == 0:
                acc += float(loss.cpu())
            steps += 1
        hist.append(acc / max(1, (steps + 15) // 16))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4f}")
    return hist


def fold_label_scale(net: CNN, scale: float):
    """Multiply the last layer by the label scale so outputs are in nm, and
    remove the network's output for a flat wavefront (zero input) from the
    last bias, so that a perfectly corrected frame gives exactly zero and
    an integrator fed by the network has no constant drift."""
    import torch
    p = net.get_params().cpu().numpy()
    off = 0
    offs = {}
    for k in PARAM_ORDER:
        n = int(np.prod(net.shapes[k]))
        offs[k] = (off, n)
        if k in ("fw2", "fb2"):
            p[off:off + n] *= scale
        off += n
    net.set_params(torch.from_numpy(p))
    zero = torch.zeros((1, net.n_sub, net.n_sub, 4), device="cuda")
    b0 = net.forward(zero).cpu().numpy()[0].astype(np.float64)
    o, n = offs["fb2"]
    p[o:o + n] = (p[o:o + n].astype(np.float64) - b0).astype(np.float32)
    net.set_params(torch.from_numpy(p))


def save_checkpoint(path: str, net: CNN, meta: dict):
    np.savez(path, params=net.get_params().cpu().numpy(), **{k: np.asarray(v) for k, v in meta.items()})


def load_checkpoint(path: str, net: CNN) -> dict:
    import torch
    d = np.load(path, allow_pickle=False)
    net.set_params(torch.from_numpy(d["params"]))
    return {k: d[k] for k in d.files if k != "params"}


def train_reconstructor(plan, R_dev, modes: np.ndarray, pupil: np.ndarray, bank, n_frames: int, seed: int,
                        epochs: int = 4, batch: int = 256, lr: float = 1e-3, r0_range=(0.06, 0.2),
                        residuals=None, weight_floor_nm: float | None = 20.0, log=None, device="cuda"):
    """Generate the training set, train a CNN from a seeded He initialisation,
    fold the label scale and the zero-input offset; returns (net, info)."""
    import time
    t0 = time.time()
    data = make_training_set(plan, bank, R_dev, modes, pupil, n_frames, seed, r0_range=r0_range,
                             residuals=residuals, device=device)
    if weight_floor_nm is not None:
        data.set_relative_weights(weight_floor_nm)
    t_data = time.time() - t0
    net = CNN(n_sub=plan.n_sub, n_out=modes.shape[0], batch_max=batch)
    import torch
    net.set_params(torch.from_numpy(he_init(net.shapes, seed + 1)))
    t1 = time.time()
    hist = []
    for ep in range(epochs):
        hist += train(net, data, 1, batch, lr * (0.5 ** ep), seed + 10 + ep, log)
    torch.cuda.synchronize()
    t_train = time.time() - t1
    fold_label_scale(net, data.label_scale)
    info = {"frames": n_frames, "epochs": epochs, "batch": batch, "loss_history": hist,
            "target": "correction to the linear estimate, c_true - R s",
            "loss": "relative (per-frame weights, floor %s nm)" % weight_floor_nm if weight_floor_nm else "MSE",
            "label_scale_nm": data.label_scale, "data_s": round(t_data, 2), "train_s": round(t_train, 2),
            "train_frames_per_s": round(epochs * n_frames / max(t_train, 1e-9), 1)}
    del data
    return net, info


def open_loop_errors(plan, net, R_dev, modes: np.ndarray, pupil: np.ndarray, bank, n_frames: int, seed: int,
                     r0_range, device="cuda"):
    """Held-out modal reconstruction error (nm RMS over the pupil, within the
    modal subspace) of the learned (R s + f(x)) and of the linear (R s)
    reconstructor on open-loop screens."""
    import torch
    data = make_training_set(plan, bank, R_dev, modes, pupil, n_frames, seed, r0_range=r0_range,
                             corrected_fraction=0.0, label_scale=1.0, device=device)
    M = modes.shape[0]
    pred = torch.empty_like(data.y)
    for b0 in range(0, n_frames, net.batch_max):
        nb = min(net.batch_max, n_frames - b0)
        net.forward(data.x[b0:b0 + nb].contiguous(), pred[b0:b0 + nb])
    y = data.y.cpu().numpy().astype(np.float64)                 # c_true - R s, nm
    e_cnn = float(np.sqrt(np.mean(np.sum((pred.cpu().numpy() - y) ** 2, axis=1))))
    e_lin = float(np.sqrt(np.mean(np.sum(y ** 2, axis=1))))
    e_0 = float(np.sqrt(np.mean(M * data.frame_rms ** 2)))
    return {"cnn_nm": round(e_cnn, 2), "linear_nm": round(e_lin, 2), "signal_nm": round(e_0, 2),
            "frames": n_frames, "r0_range": list(r0_range)}
