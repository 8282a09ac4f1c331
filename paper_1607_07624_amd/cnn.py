"""ctypes binding of the CNN reconstructor ABI (include/pwfs_cnn.h): marshalling only."""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import load_library, _check, _stream_handle, _ptr, _need

PARAM_ORDER = ("w1", "b1", "w2", "b2", "w3", "b3", "fw1", "fb1", "fw2", "fb2")


class cnn_config(ctypes.Structure):
    _fields_ = [("n_sub", ctypes.c_int32), ("c1", ctypes.c_int32), ("c2", ctypes.c_int32),
                ("c3", ctypes.c_int32), ("hidden", ctypes.c_int32), ("n_out", ctypes.c_int32),
                ("batch_max", ctypes.c_int32), ("reserved", ctypes.c_int32)]


def _lib():
    lib = load_library()
    if not getattr(lib, "_cnn_typed", False):
        vp, i32, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float
        lib.pwfs_cnn_create.argtypes = [ctypes.POINTER(cnn_config), ctypes.POINTER(vp)]
        lib.pwfs_cnn_num_params.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        lib.pwfs_cnn_set_params.argtypes = [vp, vp, vp]
        lib.pwfs_cnn_get_params.argtypes = [vp, vp, vp]
        lib.pwfs_cnn_prepare.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp]
        lib.pwfs_cnn_forward.argtypes = [vp, vp, i32, vp, vp]
        lib.pwfs_cnn_forward_acc.argtypes = [vp, vp, i32, f32, f32, vp, vp]
        lib.pwfs_cnn_gradients.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp]
        lib.pwfs_cnn_train_step.argtypes = [vp, vp, vp, vp, i32, f32, f32, f32, f32, vp, vp]
        lib.pwfs_cnn_get_optimizer.argtypes = [vp, vp, vp, ctypes.POINTER(ctypes.c_int64), vp]
        lib.pwfs_cnn_set_optimizer.argtypes = [vp, vp, vp, ctypes.c_int64, vp]
        lib.pwfs_cnn_destroy.argtypes = [vp]
        lib.pwfs_cnn_destroy.restype = None
        for n in ("pwfs_cnn_create", "pwfs_cnn_num_params", "pwfs_cnn_set_params", "pwfs_cnn_get_params",
                  "pwfs_cnn_prepare", "pwfs_cnn_forward", "pwfs_cnn_forward_acc", "pwfs_cnn_gradients",
                  "pwfs_cnn_train_step", "pwfs_cnn_get_optimizer", "pwfs_cnn_set_optimizer"):
            getattr(lib, n).restype = ctypes.c_int
        lib._cnn_typed = True
    return lib


def param_shapes(n_sub=40, c1=32, c2=64, c3=64, hidden=2048, n_out=600):
    s3 = n_sub
    for _ in range(3):
        s3 = (s3 + 1) // 2
    flat = s3 * s3 * c3
    return {"w1": (c1, 4, 3, 3), "b1": (c1,), "w2": (c2, c1, 3, 3), "b2": (c2,), "w3": (c3, c2, 3, 3),
            "b3": (c3,), "fw1": (hidden, flat), "fb1": (hidden,), "fw2": (n_out, hidden), "fb2": (n_out,)}


def he_init(shapes: dict, seed: int) -> np.ndarray:
    """Flat FP32 parameter vector: He-normal weights, zero biases (seeded, host)."""
    rng = np.random.default_rng(seed)
    parts = []
    for k in PARAM_ORDER:
        s = shapes[k]
        if len(s) > 1:
            parts.append(rng.normal(0.0, np.sqrt(2.0 / np.prod(s[1:])), s).ravel())
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts).astype(np.float32)


class CNN:
    """pwfs_cnn_* for one network (bf16 MFMA products, FP32 master weights and Adam)."""

    def __init__(self, n_sub=40, c1=32, c2=64, c3=64, hidden=2048, n_out=600, batch_max=256):
        import torch
        self._torch = torch
        self.lib = _lib()
        self.shapes = param_shapes(n_sub, c1, c2, c3, hidden, n_out)
        self.n_sub, self.n_out, self.batch_max = n_sub, n_out, batch_max
        c = cnn_config(n_sub=n_sub, c1=c1, c2=c2, c3=c3, hidden=hidden, n_out=n_out, batch_max=batch_max,
                       reserved=0)
        h = ctypes.c_void_p()
        _check(self.lib.pwfs_cnn_create(ctypes.byref(c), ctypes.byref(h)), "pwfs_cnn_create")
        self.handle = h
        n = ctypes.c_int64()
        _check(self.lib.pwfs_cnn_num_params(h, ctypes.byref(n)), "pwfs_cnn_num_params")
        self.n_params = n.value
        self.device = torch.cuda.current_device()

    def _s(self):
        return _stream_handle(self._torch, self.device)

    def set_params(self, flat):
        t = self._torch
        flat = flat if isinstance(flat, t.Tensor) else t.from_numpy(np.ascontiguousarray(flat, np.float32))
        flat = flat.to(device="cuda", dtype=t.float32).contiguous()
        _need(flat, t, t.float32, self.n_params, "params")
        _check(self.lib.pwfs_cnn_set_params(self.handle, _ptr(flat), self._s()), "pwfs_cnn_set_params")
        t.cuda.current_stream().synchronize()

    def get_params(self):
        t = self._torch
        out = t.empty(self.n_params, dtype=t.float32, device="cuda")
        _check(self.lib.pwfs_cnn_get_params(self.handle, _ptr(out), self._s()), "pwfs_cnn_get_params")
        return out

    def forward(self, x, out=None):
        t = self._torch
        B = x.shape[0]
        _need(x, t, t.float32, B * self.n_sub * self.n_sub * 4, "x")
        if out is None:
            out = t.empty((B, self.n_out), dtype=t.float32, device=x.device)
        _need(out, t, t.float32, B * self.n_out, "out")
        _check(self.lib.pwfs_cnn_forward(self.handle, _ptr(x), B, _ptr(out), self._s()), "pwfs_cnn_forward")
        return out

    def forward_acc(self, x, out, alpha: float, beta: float):
        """out = alpha * net(x) + beta * out (in place)."""
        t = self._torch
        B = x.shape[0]
        _need(x, t, t.float32, B * self.n_sub * self.n_sub * 4, "x")
        _need(out, t, t.float32, B * self.n_out, "out")
        _check(self.lib.pwfs_cnn_forward_acc(self.handle, _ptr(x), B, float(alpha), float(beta), _ptr(out),
                                             self._s()), "pwfs_cnn_forward_acc")
        return out

    def gradients(self, x, target, weights=None, grads=None, loss=None):
        """(gradients [n_params], loss [1]); grads / loss: output tensors to
        write (new ones when None)."""
        t = self._torch
        B = x.shape[0]
        _need(x, t, t.float32, B * self.n_sub * self.n_sub * 4, "x")
        _need(target, t, t.float32, B * self.n_out, "target")
        if weights is not None:
            _need(weights, t, t.float32, B, "weights")
        g = t.empty(self.n_params, dtype=t.float32, device=x.device) if grads is None else grads
        loss = t.empty(1, dtype=t.float32, device=x.device) if loss is None else loss
        _need(g, t, t.float32, self.n_params, "grads")
        _need(loss, t, t.float32, 1, "loss")
        _check(self.lib.pwfs_cnn_gradients(self.handle, _ptr(x), _ptr(target), _ptr(weights), B, _ptr(g),
                                           _ptr(loss), self._s()), "pwfs_cnn_gradients")
        return g, loss

    def train_step(self, x, target, lr, beta1=0.9, beta2=0.999, eps=1e-8, loss=None, weights=None):
        t = self._torch
        B = x.shape[0]
        _need(x, t, t.float32, B * self.n_sub * self.n_sub * 4, "x")
        _need(target, t, t.float32, B * self.n_out, "target")
        if weights is not None:
            _need(weights, t, t.float32, B, "weights")
        _check(self.lib.pwfs_cnn_train_step(self.handle, _ptr(x), _ptr(target), _ptr(weights), B, lr, beta1, beta2,
                                            eps, _ptr(loss), self._s()), "pwfs_cnn_train_step")
        return loss

    def save(self, path: str):
        """Checkpoint: FP32 master parameters, Adam moments and step count,
        and the architecture, to an .npz file (no pickled objects)."""
        t = self._torch
        m = t.empty(self.n_params, dtype=t.float32, device="cuda")
        v = t.empty(self.n_params, dtype=t.float32, device="cuda")
        step = ctypes.c_int64()
        _check(self.lib.pwfs_cnn_get_optimizer(self.handle, _ptr(m), _ptr(v), ctypes.byref(step), self._s()),
               "pwfs_cnn_get_optimizer")
        w = self.get_params()
        arch = np.array([self.n_sub, self.shapes["w1"][0], self.shapes["w2"][0], self.shapes["w3"][0],
                         self.shapes["fb1"][0], self.n_out], np.int64)
        np.savez(path, params=w.cpu().numpy(), adam_m=m.cpu().numpy(), adam_v=v.cpu().numpy(),
                 step=np.array(step.value, np.int64), arch=arch)

    def load(self, path: str):
        """Restore a checkpoint written by save() into this network (same
        architecture): parameters, Adam moments and step count."""
        t = self._torch
        with np.load(path, allow_pickle=False) as f:
            arch = [int(a) for a in f["arch"]]
            mine = [self.n_sub, self.shapes["w1"][0], self.shapes["w2"][0], self.shapes["w3"][0],
                    self.shapes["fb1"][0], self.n_out]
            if arch != mine:
                raise ValueError(f"checkpoint architecture {arch} differs from the network's {mine}")
            w, m, v, step = f["params"], f["adam_m"], f["adam_v"], int(f["step"])
        self.set_params(w)
        md = t.from_numpy(np.ascontiguousarray(m, np.float32)).cuda()
        vd = t.from_numpy(np.ascontiguousarray(v, np.float32)).cuda()
        _need(md, t, t.float32, self.n_params, "adam_m")
        _need(vd, t, t.float32, self.n_params, "adam_v")
        _check(self.lib.pwfs_cnn_set_optimizer(self.handle, _ptr(md), _ptr(vd), step, self._s()),
               "pwfs_cnn_set_optimizer")
        t.cuda.current_stream().synchronize()

    def close(self):
        if getattr(self, "handle", None):
            self.lib.pwfs_cnn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def prepare(pupils, ref_pupils, valid, out=None):
    """Network input [B, S, S, 4] from pupils [B, 4, S, S], ref [4, S, S], valid int32 [nv] (device)."""
    import torch
    lib = _lib()
    B, _, S, _ = pupils.shape
    nv = valid.numel()
    _need(pupils, torch, torch.float32, B * 4 * S * S, "pupils")
    _need(ref_pupils, torch, torch.float32, 4 * S * S, "ref_pupils")
    _need(valid, torch, torch.int32, nv, "valid")
    if out is None:
        out = torch.empty((B, S, S, 4), dtype=torch.float32, device=pupils.device)
    _need(out, torch, torch.float32, B * S * S * 4, "out")
    _check(lib.pwfs_cnn_prepare(_ptr(pupils), _ptr(ref_pupils), _ptr(valid), nv, B, S, _ptr(out),
                                _stream_handle(torch, pupils.device)), "pwfs_cnn_prepare")
    return out
