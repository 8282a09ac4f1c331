"""Write the FP64 oracle's calibration and closed-loop residuals at the
LBT-like shapes (N 640, P 160, K 48, 40 x 40 subapertures, 600 KL modes).

Calls only `oracle/` and the shared input generators in `synth/`; nothing
here touches the HIP library.  Run from the repository root:

    python tests/golden/make_cfg2_loop_golden.py [--procs 8]

Outputs (next to this script):
  cfg2_oracle_im_fp32.npy   interaction matrix [2 n_valid, 600], push-pull
                            with 10 nm on each FP32-rounded KL mode (the modal
                            reconstructor's calibration, Sec. 4 text, Tab. 1
                            "modalrec"), rounded to FP32: this rounded matrix
                            is the shared calibration both loops use
                            (R = its FP64 pseudo-inverse, nothing truncated).
  cfg2_oracle_loops.json    per-step piston-removed residual RMS (nm) of the
                            oracle's integrator loops (Tab. 1 "control": gain
                            0.4, delay 2; 1 ms steps; residual over steps
                            t >= 50, the camera's start time): the benchmark
                            loop (r0 0.12 m, 1000 steps) and the precision
                            study loops (r0 of each seed's screen, 500 steps),
                            plus a fingerprint of the KL basis they used.

About 50 minutes on 8 host cores (one FFT thread per process).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

os.environ.setdefault("ORACLE_FFT_WORKERS", "1")
HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
from concurrent.futures import ProcessPoolExecutor  # noqa: E402

import oracle  # noqa: E402
from oracle import recon as orecon  # noqa: E402
from synth.configs import (CFG2, ATMO2, CFG4_R0_RANGE, CFG4_LOOP_SEEDS, CFG4_LOOP_STEPS, CFG2_LOOP_SEED,  # noqa: E402
                           CFG2_LOOP_STEPS, PUSH_PULL_NM, LOOP_GAIN, LOOP_DELAY, LOOP_SETTLE_STEPS, N_KL_MODES)
from synth.kl import kl_modes  # noqa: E402
from synth.screens import frozen_flow_sequence, cfg4_loop_sequence  # noqa: E402

IM_PATH = os.path.join(HERE, "cfg2_oracle_im_fp32.npy")
JSON_PATH = os.path.join(HERE, "cfg2_oracle_loops.json")


def basis_fingerprint(modes: np.ndarray, A: np.ndarray) -> np.ndarray:
    """Mean over the pupil pixels of each mode times a seeded Gaussian field:
    a basis computed elsewhere is the same one iff these agree."""
    w = np.random.default_rng(7).standard_normal(int((A > 0).sum()))
    flat = modes.reshape(modes.shape[0], -1)[:, A.ravel() > 0].astype(np.float64)
    return flat @ w / w.size


def _modes():
    A = oracle.pupil_amplitude(CFG2.n_pupil, CFG2.obstruction)
    return kl_modes(A, CFG2.pixel_m, ATMO2.L0_m, N_KL_MODES).astype(np.float32), A


def _im_columns(idx):
    modes, _ = _modes()
    orc = oracle.Oracle(CFG2)
    meas = lambda r: orc.measure(r)[1]
    out = orecon.interaction_matrix(meas, modes[idx].astype(np.float64), PUSH_PULL_NM)
    print(f"  IM columns {idx[0]}..{idx[-1]} done", flush=True)
    return out


def _loop(job):
    name, seq = job
    modes, A = _modes()
    IM = np.load(IM_PATH).astype(np.float64)
    R, _ = orecon.pseudo_inverse(IM)
    orc = oracle.Oracle(CFG2)
    t0 = time.time()
    rms, _ = orecon.closed_loop(lambda r: orc.measure(r)[1], seq, modes.astype(np.float64), R,
                                LOOP_GAIN, LOOP_DELAY, A)
    print(f"  loop {name}: {orecon.loop_residual_nm(rms, LOOP_SETTLE_STEPS):.4f} nm "
          f"({time.time() - t0:.0f} s)", flush=True)
    return name, rms


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--skip-im", action="store_true", help="reuse the stored interaction matrix")
    args = ap.parse_args()
    modes, A = _modes()
    if not args.skip_im:
        t0 = time.time()
        chunks = [list(c) for c in np.array_split(np.arange(N_KL_MODES), 4 * args.procs)]
        with ProcessPoolExecutor(args.procs) as ex:
            cols = list(ex.map(_im_columns, chunks))
        IM = np.concatenate(cols, axis=1)
        np.save(IM_PATH, IM.astype(np.float32))
        print(f"IM {IM.shape} in {time.time() - t0:.0f} s", flush=True)
    IM = np.load(IM_PATH).astype(np.float64)
    sig = np.linalg.svd(IM, compute_uv=False)

    jobs = [(f"cfg2_r0_0.12_seed{CFG2_LOOP_SEED}",
             frozen_flow_sequence(CFG2, ATMO2, CFG2_LOOP_STEPS, seed=CFG2_LOOP_SEED))]
    r0s = {}
    for s in CFG4_LOOP_SEEDS:
        seq, r0 = cfg4_loop_sequence(CFG2, ATMO2, s, CFG4_LOOP_STEPS, CFG4_R0_RANGE)
        jobs.append((f"cfg4_seed{s}", seq))
        r0s[f"cfg4_seed{s}"] = r0
    open_loop = {name: orecon.loop_residual_nm(
        np.array([orecon.residual_rms_nm(f.astype(np.float64), A) for f in seq]), LOOP_SETTLE_STEPS)
        for name, seq in jobs}
    with ProcessPoolExecutor(min(args.procs, len(jobs))) as ex:
        loops = dict(ex.map(_loop, jobs))
    out = {
        "about": "FP64 oracle: push-pull IM (10 nm) on the 600 FP32-rounded KL modes, rounded to FP32; "
                 "R = full-SVD pseudo-inverse of that matrix in FP64; integrator loops gain 0.4, delay 2; "
                 "rms[t] = piston-removed residual RMS over the pupil in nm; residual = RMS over t >= 50. "
                 "Written by tests/golden/make_cfg2_loop_golden.py.",
        "n_slopes": int(IM.shape[0]), "n_modes": int(IM.shape[1]),
        "im_singular_values_max_min": [float(sig[0]), float(sig[-1])],
        "kl_fingerprint": basis_fingerprint(modes, A).tolist(),
        "loops": {name: {"r0_m": r0s.get(name, ATMO2.r0_m),
                         "steps": int(len(loops[name])),
                         "sequence": ("frozen_flow_sequence(CFG2, ATMO2, %d, seed=%d)" % (CFG2_LOOP_STEPS, CFG2_LOOP_SEED)
                                      if name.startswith("cfg2") else
                                      "cfg4_loop_sequence(CFG2, ATMO2, %s, %d)" % (name[9:], CFG4_LOOP_STEPS)),
                         "open_loop_nm": open_loop[name],
                         "residual_nm": orecon.loop_residual_nm(loops[name], LOOP_SETTLE_STEPS),
                         "rms_nm": [float(v) for v in loops[name]]}
                  for name, _ in jobs},
    }
    with open(JSON_PATH, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {JSON_PATH}", flush=True)


if __name__ == "__main__":
    main()
