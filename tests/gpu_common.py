"""Shared helpers of the GPU tests (inputs and comparisons, no arithmetic of the method)."""
import sys

import numpy as np


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a visible HIP device")
    return torch


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_max(a, b):
    """max |a - b| / max |b|: a per-element bound next to the relative L2."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


SLOPE_TOL = 1e-5     # the sensor's slope bound (relative L2, and max error over max |slope|)
PUPIL_TOL = 2e-6     # binned pupils: FP32 accumulation over modulation points and bins


def check_frame(tag, s, s_o, p=None, p_o=None, slope_tol=SLOPE_TOL, pupil_tol=PUPIL_TOL):
    """Relative L2 and per-element (max |error| / max |reference|) gates of one
    frame's slopes and, when given, pupils; prints both and returns the slope
    relative L2."""
    e_s, m_s = rel_l2(s, s_o), rel_max(s, s_o)
    msg = f"[gpu]   {tag}: slope rel err {e_s:.3e} (max {m_s:.3e})"
    ok = e_s <= slope_tol and m_s <= slope_tol
    if p is not None:
        e_p, m_p = rel_l2(p, p_o), rel_max(p, p_o)
        msg += f"  pupil rel err {e_p:.3e} (max {m_p:.3e})"
        ok = ok and e_p <= pupil_tol and m_p <= pupil_tol
    say(msg)
    assert ok, msg
    return e_s
