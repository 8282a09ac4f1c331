"""FP64 reference of the learned (CNN) modal reconstructor: forward,
hand-written backward, MSE loss and Adam.

Test infrastructure only (see the package docstring).

The network maps the four binned pupil images to modal (KL) coefficients,
the same output as the paper's modal reconstructor (Sec. 4, Tab. 1
"modalrec", Tab. 2 rec.in_slopes -> out_modes), so either can feed the
integrator.  Architecture (fixed here, the paper has no learned part):
  input  [B, S, S, 4]  (NHWC; S = 40 at the LBT-like geometry)
  conv 3x3 stride 2 pad 1, 4 -> 32, ReLU      -> [B, 20, 20, 32]
  conv 3x3 stride 2 pad 1, 32 -> 64, ReLU     -> [B, 10, 10, 64]
  conv 3x3 stride 2 pad 1, 64 -> 64, ReLU     -> [B, 5, 5, 64]
  flatten in (y, x, c) order                 -> [B, 1600]
  fully connected 1600 -> 2048, ReLU
  fully connected 2048 -> 600                 (modal coefficients / label scale)
Parameters: conv weights [Cout, Cin, 3, 3], biases [Cout]; fc weights
[Nout, Nin], biases [Nout].  The flat parameter vector concatenates
w1, b1, w2, b2, w3, b3, fw1, fb1, fw2, fb2 in that order, C-contiguous.
Loss: mean over all outputs of w_b (prediction - target)^2 with an optional
per-frame weight w_b (1 by default).
Adam: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np

PARAM_ORDER = ("w1", "b1", "w2", "b2", "w3", "b3", "fw1", "fb1", "fw2", "fb2")


def param_shapes(S: int = 40, c_in: int = 4, chans=(32, 64, 64), hidden: int = 2048, n_out: int = 600):
    c1, c2, c3 = chans
    s3 = S
    for _ in range(3):
        s3 = (s3 + 1) // 2
    flat = s3 * s3 * c3
    return {"w1": (c1, c_in, 3, 3), "b1": (c1,), "w2": (c2, c1, 3, 3), "b2": (c2,),
            "w3": (c3, c2, 3, 3), "b3": (c3,), "fw1": (hidden, flat), "fb1": (hidden,),
            "fw2": (n_out, hidden), "fb2": (n_out,)}


def flatten_params(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], np.float64).ravel() for k in PARAM_ORDER])


def unflatten_params(v: np.ndarray, shapes: dict) -> dict:
    out, o = {}, 0
    for k in PARAM_ORDER:
        n = int(np.prod(shapes[k]))
        out[k] = np.asarray(v[o:o + n], np.float64).reshape(shapes[k])
        o += n
    assert o == v.size
    return out


def conv_forward(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[b, yo, xo, o] = b[o] + sum_{c, ky, kx} w[o, c, ky, kx] x[b, 2 yo + ky - 1, 2 xo + kx - 1, c]
    with zeros outside x (stride 2, padding 1)."""
    B, H, W, C = x.shape
    Ho, Wo = (H + 1) // 2, (W + 1) // 2
    xp = np.zeros((B, H + 2, W + 2, C))
    xp[:, 1:H + 1, 1:W + 1] = x
    y = np.broadcast_to(b, (B, Ho, Wo, w.shape[0])).copy()
    for ky in range(3):
        for kx in range(3):
            xs = xp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2, :]
            y += xs @ w[:, :, ky, kx].T
    return y


def conv_backward(x: np.ndarray, w: np.ndarray, dy: np.ndarray):
    """Gradients (dx, dw, db) of conv_forward for the upstream gradient dy."""
    B, H, W, C = x.shape
    Ho, Wo = dy.shape[1], dy.shape[2]
    xp = np.zeros((B, H + 2, W + 2, C))
    xp[:, 1:H + 1, 1:W + 1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    dyf = dy.reshape(-1, dy.shape[3])
    for ky in range(3):
        for kx in range(3):
            xs = xp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2, :]
            dw[:, :, ky, kx] = dyf.T @ xs.reshape(-1, C)
            dxp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2, :] += dy @ w[:, :, ky, kx]
    return dxp[:, 1:H + 1, 1:W + 1], dw, dyf.sum(axis=0)


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a32 = np.ascontiguousarray(a, np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(p: dict, x: np.ndarray):
    """(prediction [B, n_out], cache) for NHWC input x, exact FP64."""
    a1 = np.maximum(conv_forward(x, p["w1"], p["b1"]), 0.0)
    a2 = np.maximum(conv_forward(a1, p["w2"], p["b2"]), 0.0)
    a3 = np.maximum(conv_forward(a2, p["w3"], p["b3"]), 0.0)
    f = a3.reshape(a3.shape[0], -1)
    h = np.maximum(f @ p["fw1"].T + p["fb1"], 0.0)
    out = h @ p["fw2"].T + p["fb2"]
    return out, (x, a1, a2, a3, f, h)


def mse(pred: np.ndarray, target: np.ndarray, weights=None):
    """(loss, d loss / d pred); weights [B] scale each frame's squared error."""
    d = pred - target
    w = np.ones(d.shape[0]) if weights is None else np.asarray(weights, np.float64)
    return float(np.mean(w[:, None] * d * d)), 2.0 * w[:, None] * d / d.size


def backward(p: dict, cache, dout: np.ndarray) -> dict:
    """Parameter gradients for the upstream gradient dout (d loss / d prediction)."""
    x, a1, a2, a3, f, h = cache
    g = {}
    g["fw2"] = dout.T @ h
    g["fb2"] = dout.sum(axis=0)
    dh = (dout @ p["fw2"]) * (h > 0)
    g["fw1"] = dh.T @ f
    g["fb1"] = dh.sum(axis=0)
    da3 = (dh @ p["fw1"]).reshape(a3.shape) * (a3 > 0)
    da2, g["w3"], g["b3"] = conv_backward(a2, p["w3"], da3)
    da2 = da2 * (a2 > 0)
    da1, g["w2"], g["b2"] = conv_backward(a1, p["w2"], da2)
    da1 = da1 * (a1 > 0)
    _, g["w1"], g["b1"] = conv_backward(x, p["w1"], da1)
    return g


def loss_and_grads(p: dict, x: np.ndarray, target: np.ndarray, weights=None):
    pred, cache = forward(p, x)
    loss, dout = mse(pred, target, weights)
    return loss, backward(p, cache, dout), pred


def adam_step(w, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step count t >= 1); returns new (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def network_input(pupils: np.ndarray, ref_pupils: np.ndarray, valid: np.ndarray) -> np.ndarray:
    """NHWC network input [B, S, S, 4] from binned pupils [B, 4, S, S]:
    each frame divided by its mean total flux over the valid subapertures,
    minus the flat-wavefront pupils normalised the same way, zero outside
    the valid subapertures."""
    pupils = np.asarray(pupils, np.float64)
    B, _, S, _ = pupils.shape
    mask = np.zeros(S * S)
    mask[valid] = 1.0
    mask = mask.reshape(S, S)

    def norm(p):
        tot = p.reshape(p.shape[0], 4, -1)[:, :, valid].sum(axis=1).mean(axis=1)
        return p / tot[:, None, None, None]

    x = (norm(pupils) - norm(np.asarray(ref_pupils, np.float64)[None])) * mask
    return np.transpose(x, (0, 2, 3, 1))


def kl_coefficients(opd_nm: np.ndarray, modes_nm: np.ndarray, A: np.ndarray) -> np.ndarray:
    """Modal coefficients c_i = mean over the pupil of B_i * opd (the modes are
    orthonormal with unit RMS over the pupil, so this is the projection)."""
    sel = A.ravel() > 0
    Bm = modes_nm.reshape(modes_nm.shape[0], -1)[:, sel]
    o = np.asarray(opd_nm, np.float64).reshape(np.asarray(opd_nm).shape[0], -1)[:, sel]
    return o @ Bm.T / sel.sum()
