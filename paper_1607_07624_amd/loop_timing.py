"""Step rate of the single-sensor closed loop at the LBT-like geometry
(P = 160, N = 640, K = 48, 40 x 40 subapertures, 600 KL modes, gain 0.4,
delay 2) on a frozen-flow sequence: the eager loop (library calls launched
one by one) and the graph-replayed loop, same residuals.  Run as

    python -m paper_1607_07624_amd.loop_timing [--steps 200]

which prints one JSON line (steps/s of both, and whether they agree bit
for bit).  Under `rocprofv3 --kernel-trace` the two phases are separated by
two marker launches of `recon_apply` on a 3 x 5 matrix (the scalar form of
the reconstructor kernel, which the loop itself never uses), so the
per-step kernels of each phase can be told apart.
"""
from __future__ import annotations

import argparse
import json


def measure(steps: int = 200, seed: int = 2024) -> dict:
    import numpy as np
    import torch
    from . import Plan
    from .loop import calibrate, ClosedLoop
    from synth.configs import CFG2, ATMO2, N_KL_MODES, PUSH_PULL_NM, LOOP_GAIN, LOOP_DELAY
    from synth.screens import frozen_flow_sequence
    from synth.kl import kl_modes

    dev = torch.device("cuda", torch.cuda.current_device())
    cal = Plan(CFG2, batch_max=16)
    amp = cal.pupil.astype(np.float64)
    modes = kl_modes(amp, CFG2.pixel_m, ATMO2.L0_m, N_KL_MODES).astype(np.float32)
    R, _, _ = calibrate(cal, modes, PUSH_PULL_NM, dev)
    cal.close()
    plan = Plan(CFG2, batch_max=1)
    plan.autotune(1, reps=5)
    seq = torch.from_numpy(frozen_flow_sequence(CFG2, ATMO2, steps, seed=seed)).to(dev)
    cl = ClosedLoop(plan, torch.from_numpy(modes).to(dev), R, LOOP_GAIN, LOOP_DELAY)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    cl.run(seq[:10])
    torch.cuda.synchronize()
    ev0.record()
    res_e, _ = cl.run(seq)
    ev1.record()
    torch.cuda.synchronize()
    eager_ms = ev0.elapsed_time(ev1)
    from ._lib import recon_apply
    mk = torch.ones((3, 5), device=dev)
    mo = torch.zeros((1, 3), device=dev)
    for _ in range(2):                # marker between the phases
        recon_apply(mk, torch.ones((1, 5), device=dev), 1.0, 0.0, mo)
    torch.cuda.synchronize()
    ev0.record()
    res_g, _ = cl.run_graph(seq)
    ev1.record()
    torch.cuda.synchronize()
    graph_ms = ev0.elapsed_time(ev1)
    same = bool(torch.equal(res_e, res_g))
    plan.close()
    return {"steps": steps, "eager_steps_per_s": round(steps / (eager_ms * 1e-3), 1),
            "graph_steps_per_s": round(steps / (graph_ms * 1e-3), 1), "graph_equals_eager": same}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=200)
    args = ap.parse_args()
    print(json.dumps(measure(args.steps)), flush=True)


if __name__ == "__main__":
    main()
