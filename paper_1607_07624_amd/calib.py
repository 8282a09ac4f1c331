"""Tagged calibration data on disk (the paper's calibration manager, Sec. 2
and Sec. 4: calibration products are written once under a tag and read back
by later runs instead of being measured again).

A calibration file is an ``.npz`` of plain arrays (no pickled objects; it is
read with ``numpy.load(allow_pickle=False)``) holding its tag, a key and the
arrays.  The key is a SHA-256 over everything the arrays depend on: the
sensor configuration, the pupil amplitude, the valid-subaperture list, the
modal basis and the push-pull amplitude.  A file whose key differs from the
one asked for is stale and is never returned, so a changed geometry, basis
or valid list always leads to a new calibration.

``calibrate_cached`` stores, under one tag, what a closed loop needs to start
without measuring: the valid list, the slope reference, the KL basis, the
interaction matrix, the reconstructor and its singular values.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

FORMAT = "pwfs-calib-1"


def _feed(h, name: str, v) -> None:
    h.update(name.encode() + b"\0")
    if isinstance(v, np.ndarray) or hasattr(v, "__array__"):
        a = np.ascontiguousarray(np.asarray(v))
        h.update(f"{a.dtype.str}{a.shape}".encode())
        h.update(a.tobytes())
    else:
        h.update(json.dumps(v, sort_keys=True, default=str).encode())
    h.update(b"\1")


def config_hash(cfg, **parts) -> str:
    """Hex SHA-256 of a sensor configuration (a dataclass with as_dict(), or a
    dict) and named extra parts (arrays by dtype, shape and bytes; other
    values by their JSON form), independent of the order the parts are given."""
    h = hashlib.sha256(FORMAT.encode())
    _feed(h, "cfg", cfg.as_dict() if hasattr(cfg, "as_dict") else dict(cfg))
    for k in sorted(parts):
        _feed(h, k, parts[k])
    return h.hexdigest()


class CalibrationStore:
    """A directory of tagged calibration files, ``<root>/<tag>.npz``."""

    def __init__(self, root: str):
        self.root = os.path.abspath(root)

    def path(self, tag: str) -> str:
        if not tag or any(c in tag for c in "/\\\0") or tag.startswith("."):
            raise ValueError(f"bad calibration tag {tag!r}")
        return os.path.join(self.root, tag + ".npz")

    def tags(self) -> list:
        if not os.path.isdir(self.root):
            return []
        return sorted(f[:-4] for f in os.listdir(self.root) if f.endswith(".npz"))

    def save(self, tag: str, key: str, **arrays) -> str:
        """Write the arrays under tag with key (atomically: a reader sees the
        old file or the new one, never half of one).  Returns the path."""
        for name in arrays:
            if name.startswith("_"):
                raise ValueError("array names starting with '_' are reserved")
        os.makedirs(self.root, exist_ok=True)
        p = self.path(tag)
        tmp = p + f".tmp{os.getpid()}"
        with open(tmp, "wb") as f:
            np.savez(f, _format=np.array(FORMAT), _tag=np.array(tag), _key=np.array(key),
                     **{k: np.asarray(v) for k, v in arrays.items()})
        os.replace(tmp, p)
        return p

    def key_of(self, tag: str):
        """The key stored under tag, or None if there is no such file."""
        p = self.path(tag)
        if not os.path.exists(p):
            return None
        with np.load(p, allow_pickle=False) as z:
            return str(z["_key"])

    def load(self, tag: str, key: str):
        """The arrays stored under tag if its key equals key, else None (no
        file, another format or a stale key)."""
        p = self.path(tag)
        if not os.path.exists(p):
            return None
        with np.load(p, allow_pickle=False) as z:
            if "_format" not in z.files or str(z["_format"]) != FORMAT or str(z["_key"]) != key:
                return None
            return {k: z[k] for k in z.files if not k.startswith("_")}


def recmat_key(plan, modes: np.ndarray, eps_nm: float) -> str:
    """Key of a modal reconstructor measured on plan: its configuration,
    pupil amplitude and valid list, the basis and the push-pull amplitude."""
    return config_hash(plan.cfg, pupil=plan.pupil.astype(np.float32), valid=plan.valid,
                       modes=np.ascontiguousarray(modes, np.float32), eps_nm=float(eps_nm),
                       kind="push-pull IM, full-SVD pseudo-inverse")


def calibrate_cached(plan, modes: np.ndarray, eps_nm: float, store: CalibrationStore, tag: str = "recmat",
                     device="cuda"):
    """Reconstructor of plan for the basis modes [M, P, P]: read from store
    under tag when its key matches, else measured (loop.calibrate) and
    written there.  Returns (R as a float32 device tensor [M, n_slopes], IM
    [n_slopes, M] FP64, singular values FP64, hit)."""
    import torch
    from .loop import calibrate
    modes = np.ascontiguousarray(modes, np.float32)
    key = recmat_key(plan, modes, eps_nm)
    got = store.load(tag, key)
    if got is not None:
        R = torch.from_numpy(np.ascontiguousarray(got["R"], np.float32)).to(device)
        return R, got["IM"], got["sigma"], True
    R, IM, sig = calibrate(plan, modes, eps_nm, device)
    store.save(tag, key, R=R.cpu().numpy(), IM=IM, sigma=sig, valid=plan.valid, s_ref=plan.s_ref,
               modes=modes, eps_nm=np.float64(eps_nm), config=np.array(json.dumps(plan.cfg.as_dict())))
    return R, IM, sig, False
