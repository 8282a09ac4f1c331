"""Stored FP64-oracle calibration and closed-loop residuals at the LBT-like
shapes (written by tests/golden/make_cfg2_loop_golden.py, which calls only
the oracle and the shared input generators), and the KL basis they refer to."""
import json
import os

import numpy as np

import oracle
from synth.configs import CFG2, ATMO2, N_KL_MODES
from synth.kl import kl_modes

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
IM_PATH = os.path.join(GOLDEN, "cfg2_oracle_im_fp32.npy")
JSON_PATH = os.path.join(GOLDEN, "cfg2_oracle_loops.json")


def load():
    """(oracle IM [2 nv, 600] float64 of the stored FP32 values, loop record)."""
    with open(JSON_PATH) as f:
        rec = json.load(f)
    return np.load(IM_PATH).astype(np.float64), rec


def modes_checked(rec):
    """The 600 FP32 KL modes of the LBT-like pupil, after checking that this
    machine computes the basis the stored values were computed with (same
    modes and signs: the fingerprint agrees to 1e-8 against entries of ~7e-3)."""
    A = oracle.pupil_amplitude(CFG2.n_pupil, CFG2.obstruction)
    modes = kl_modes(A, CFG2.pixel_m, ATMO2.L0_m, N_KL_MODES).astype(np.float32)
    w = np.random.default_rng(7).standard_normal(int((A > 0).sum()))
    fp = modes.reshape(N_KL_MODES, -1)[:, A.ravel() > 0].astype(np.float64) @ w / w.size
    diff = float(np.abs(fp - np.asarray(rec["kl_fingerprint"])).max())
    assert diff <= 1e-8, f"KL basis differs from the stored one (fingerprint max diff {diff:.3e})"
    return modes, A


def loop_errors(rms_gpu, rms_oracle, settle):
    """(worst per-step relative difference, relative difference of the
    residual over t >= settle)."""
    rms_gpu = np.asarray(rms_gpu, np.float64)
    rms_oracle = np.asarray(rms_oracle, np.float64)
    worst = float(np.max(np.abs(rms_gpu - rms_oracle) / rms_oracle))
    tg = float(np.sqrt(np.mean(rms_gpu[settle:] ** 2)))
    to = float(np.sqrt(np.mean(rms_oracle[settle:] ** 2)))
    return worst, abs(tg - to) / to, tg, to
