"""Benchmark of the modulated pyramid sensor path on one MI355X.

A step is one pass of the whole path over a batch of 16 independent seeded
von Karman screens at the LBT-like geometry (P = 160 pupil pixels, 640-point
FFT grid, 48 modulation points, 40 x 40 subapertures, 600 KL modes):
pwfs_measure (row pass, column pass, slopes) followed by recon_apply with
the calibrated 600 x 2544 reconstructor.  Inputs are resident in HBM before
the timed region.  Prints one JSON line.

Besides throughput the line carries
  roofline      the column-pass kernel (the dominant one) against the FP32
                vector peak, from its algorithmic flop count and its event-
                timed average duration inside the timed region;
  cpu_baseline  the FP64 oracle timed on the host's cores on a small sample
                of the same frames;
  loop          the 1000-step frozen-flow closed loop (integrator gain 0.4,
                delay 2) run on the GPU: residual nm RMS and steps/s.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np

PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector peak (256 CU x 2.4 GHz x 256 flop/clk)
PEAK_HBM_GBS = 8000.0

# HBM bytes per 16-frame column-pass launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs
# (KiB per dispatch, scaled by the copy-kernel factors 2.0 / 1.0; summary and commands in
# profiles/pwfs_measure_n640_p160_k48_b16.md), one entry per work split (x-tilt chunk,
# modulation chunk).  Valid only for the sources with these hashes (the kernels and the plan's
# modulation order); reported as null otherwise.
COUNTER_TRAFFIC = {
    "sources_sha1": {"pwfs_kernels.hip": "57b9b0cae508d6d627e16137dff991878c3bb183",
                     "pwfs_field.h": "bc1faa09406794b7ad671c337fa21b1f47710d8a",
                     "pwfs_common.h": "3096fe01bd7ba8d5172249619ee3af04487ad813",
                     "pwfs_dft.h": "2311b455e0848ccf3b2b36c948f8cf8f42218515",
                     "pwfs_api.cpp": "6ea1b5489dff398679f44044805abaa43565d733"},
    "batch": 16,
    "col_pass_kib": {(3, 2): (81209.6, 9602.6), (3, 4): (81629.2, 4800.0), (3, 6): (81709.9, 3200.0)},
}


def counter_traffic(batch, schedule):
    import hashlib
    csrc = os.path.join(ROOT, "paper_1607_07624_amd", "csrc")
    for name, h in COUNTER_TRAFFIC["sources_sha1"].items():
        with open(os.path.join(csrc, name), "rb") as f:
            if hashlib.sha1(f.read()).hexdigest() != h:
                return None
    kib = COUNTER_TRAFFIC["col_pass_kib"].get(tuple(schedule)) if batch == COUNTER_TRAFFIC["batch"] else None
    return None if kib is None else (kib[0] * 2.0 + kib[1] * 1.0) * 1024


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# --- algorithmic flop count of the HIP line operator -----------------------
_RADIX_FLOPS = {1: 0, 2: 4, 3: 16, 4: 16, 5: 48}


def _first_radix(n):
    if n % 4 == 0 and n != 8:
        return 4
    for r in (2, 3, 5):
        if n % r == 0:
            return r
    return n


def _coprime_part(n):
    for p in range(2, n + 1):
        if n % p == 0:
            q = p
            while n % (q * p) == 0:
                q *= p
            return 0 if q == n else q
    return 0


def dft_flops(E: int) -> int:
    """Real flops of the in-register DFT of length E: the twiddle-free
    prime-factor split E = N1 N2 for coprime factors, else mixed-radix
    decimation in time (trivial twiddles free)."""
    N1 = _coprime_part(E)
    if N1:
        N2 = E // N1
        return N1 * dft_flops(N2) + N2 * dft_flops(N1)
    R = _first_radix(E)
    Q = E // R
    if Q == 1:
        return _RADIX_FLOPS[R]
    tw = sum(6 for r in range(R) for k in range(Q) if ((r * k) % E) * 4 % E != 0)
    return R * dft_flops(Q) + Q * _RADIX_FLOPS[R] + tw


def line_flops(P: int, intensity: bool) -> int:
    """Flops of one 1-D pyramid line operator (two half-band projections of
    length P in four-step form, input twist, output twiddles, y_L = f - y_H,
    plus |E|^2 accumulation in the column pass)."""
    E = P // 4
    projection = 4 * (2 * dft_flops(E) + 16 * E)     # 4 lanes: DFT_E, 3-tap mix (two complex MACs + v), IDFT_E
    f = 6 * P                                         # tilt ramp times input
    twist = 2 * 6 * P
    out = 2 * 6 * P + 2 * P + 2 * P                   # output twiddles, sum of the two halves, f - y_H
    acc = 2 * 2 * P * 2 if intensity else 0           # |.|^2 + accumulate, both windows
    return 2 * projection + f + twist + out + acc


def fft_pair_flops(N: int) -> float:
    """Algorithmic flops of one line of the separable pyramid operator: a
    forward and an inverse N-point FFT at 5 N log2 N each."""
    return 2 * 5 * N * float(np.log2(N))


def line_flops16(P: int, intensity: bool) -> int:
    """Same operator for long lines (P = 16 E, a projection on 16 lanes): per
    lane DFT_E and its inverse, the subgroup twiddle and its conjugate, the two
    radix-2 DPP stages of DFT_4 each way and the 3-tap mix."""
    E = P // 16
    projection = 16 * (2 * dft_flops(E) + 36 * E)
    f = 6 * P
    twist = 2 * 6 * P
    out = 2 * 6 * P + 2 * P + 2 * P
    acc = 2 * 2 * P * 2 if intensity else 0
    return 2 * projection + f + twist + out + acc


def strehl_stats(cam, res, P, settle):
    """H-band image quality of a loop's residual screens res [T, P*P] (device):
    the Strehl ratio of the long-exposure PSF after the settle time (the
    centre of the integrated PSF over the frame count, through the PSF camera;
    it equals the mean of the frames' Strehl ratios, checked here)."""
    import torch
    T = res.shape[0]
    r = res.view(T, P, P)[settle:].contiguous()
    _, sr = cam.compute(r, want_psf=False)
    le, _ = cam.compute(r, accumulate=True)
    N = cam.n_image
    torch.cuda.synchronize()
    s_long = float(le[N // 2, N // 2]) / (T - settle)
    assert abs(s_long - float(sr.double().mean())) <= 1e-4
    return {"strehl_h": round(s_long, 4)}


def median_of_repeats(step, calls, frames_per_call, ev0, ev1, n=5):
    """Median, min and max over n repeats of `calls` back-to-back calls, each
    bracketed by events on the current stream."""
    import torch
    ms = []
    for _ in range(n):
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(calls):
            step()
        ev1.record()
        torch.cuda.synchronize()
        ms.append(ev0.elapsed_time(ev1) / calls)
    ms.sort()
    med = ms[n // 2]
    return {"repeats": n, "calls_each": calls, "ms_per_call_median": round(med, 5),
            "ms_per_call_min": round(ms[0], 5), "ms_per_call_max": round(ms[-1], 5),
            "frames_per_s_median": round(frames_per_call / (med * 1e-3), 1)}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def multi_source_leg(args, log):
    """Six guide stars through three layers, sensed at 650 and 850 nm (40 m
    class geometry) by two plans captured in one HIP graph."""
    import torch
    from synth.configs import CFG3, CFG3_850, ATMO3, CFG3_LAYERS, CFG3_GS_ARCSEC
    from synth.screens import layered_opd_nm
    from paper_1607_07624_amd.multisource import MultiSourceSensor
    ns = len(CFG3_GS_ARCSEC)
    ms = MultiSourceSensor([CFG3, CFG3_850], n_sources=ns, autotune=True, reps=3)
    ms.opd.copy_(torch.from_numpy(layered_opd_nm(CFG3, ATMO3, CFG3_LAYERS, CFG3_GS_ARCSEC, seed=7)))
    ms.capture()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = args.multi_reps
    for _ in range(3):
        ms.measure()
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        ms.measure()
    ev1.record()
    torch.cuda.synchronize()
    graph_ms = ev0.elapsed_time(ev1) / reps
    ev0.record()
    for _ in range(reps):
        ms.measure_eager()
    ev1.record()
    torch.cuda.synchronize()
    eager_ms = ev0.elapsed_time(ev1) / reps
    kernels = []
    for p, cfg in zip(ms.plans, (CFG3, CFG3_850)):
        p.timing_enable(True)
        for _ in range(reps):
            p.measure_into(ms.opd, None, ms.slopes[0] if p is ms.plans[0] else ms.slopes[1])
        kt = p.timing_read()
        p.timing_enable(False)
        n = kt["slices"]
        col_ms = kt["col_ms"] / n
        lines = cfg.n_mod * 2 * cfg.n_pupil * ns
        kernels.append({"wavelength_nm": round(cfg.wavelength_m * 1e9), "row_ms": round(kt["row_ms"] / n, 4),
                        "col_ms": round(col_ms, 4), "slopes_ms": round(kt["slopes_ms"] / n, 4),
                        "col_tflops": round(lines * fft_pair_flops(cfg.n_fft) / (col_ms * 1e-3) / 1e12, 2),
                        "col_issued_tflops": round(lines * line_flops16(cfg.n_pupil, True) / (col_ms * 1e-3) / 1e12, 2)})
    for k in kernels:
        k["col_frac_of_fp32_peak"] = round(k["col_tflops"] / PEAK_FP32_TFLOPS, 4)
    cpu = None
    if not args.no_cpu:
        # The FP64 oracle on the host cores for one 650 nm frame of the same batch.
        import oracle
        orc = oracle.Oracle(CFG3)
        o = ms.opd[0].cpu().numpy().astype(np.float64)
        t0 = time.perf_counter()
        orc.measure(o)
        dt = time.perf_counter() - t0
        cpu = {"value": round(1.0 / dt, 4), "unit": "sensor frames/s", "cores": len(os.sched_getaffinity(0)),
               "kind": "oracle", "sample": "1 frame (650 nm, guide star 0), FP64 literal 2-D route"}
    out = {"workload": "40 m class: N=1920, P=480, K=64, b=5 (7232 valid); 6 guide stars at 45 arcsec, "
                       "3 layers (0/5/12 km), 650 + 850 nm",
           "cpu_baseline": cpu,
           "sensor_frames_per_call": 2 * ns, "graph_ms": round(graph_ms, 4), "eager_ms": round(eager_ms, 4),
           "sensor_frames_per_s": round(2 * ns / (graph_ms * 1e-3), 1),
           "schedules": [{k: v for k, v in s_.items() if k in ("a_chunk", "k_chunk")} for s_ in ms.schedules],
           "kernels": kernels}
    ms.close()
    log(f"multi-source {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--seed", type=int, default=0, help="first screen seed of the benchmark frames")
    ap.add_argument("--jsonl", type=str, default=None, help="also append the result line (with argv) to this file")
    ap.add_argument("--calib-dir", type=str, default=None,
                    help="tagged calibration cache: reuse the reconstructor stored there for this configuration")
    ap.add_argument("--cpu-frames", type=int, default=6)
    ap.add_argument("--cpu-frames-1core", type=int, default=2)
    ap.add_argument("--repeat-frames", type=int, default=2000,
                    help="frames per repeat of the median-of-5 timing (B = 16 and B = 1); 0 skips it "
                         "(counter runs: every dispatch is then instrumented)")
    ap.add_argument("--loop-steps", type=int, default=1000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-loop", action="store_true")
    ap.add_argument("--no-cnn", action="store_true", help="skip training and evaluating the learned reconstructor")
    ap.add_argument("--cnn-frames", type=int, default=200000)
    ap.add_argument("--cnn-epochs", type=int, default=4)
    ap.add_argument("--no-autotune", action="store_true", help="keep the library's default work split")
    ap.add_argument("--no-multi", action="store_true", help="skip the multi-source 40 m class leg")
    ap.add_argument("--multi-reps", type=int, default=20)
    ap.add_argument("--schedule", type=str, default=None,
                    help="A,K: fix the work split (x-tilt chunk, modulation chunk) instead of autotuning")
    ap.add_argument("--random-R", action="store_true",
                    help="profiling runs: skip calibration, use a random reconstructor of the same shape")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="after the timed region, one device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures a single GPU; --gpus {args.gpus} is not supported "
              "(the path would shard by independent frames, sources or modulation points with no exchange)",
              file=sys.stderr, flush=True)
        sys.exit(2)

    import torch
    import paper_1607_07624_amd as pw
    from paper_1607_07624_amd.loop import calibrate, ClosedLoop, BatchedLoop, residual_rms_nm
    from synth.configs import CFG2, ATMO2, CFG4_R0_RANGE, N_KL_MODES, PUSH_PULL_NM, LOOP_GAIN, \
        LOOP_DELAY, LOOP_SETTLE_STEPS
    from synth.screens import open_loop_batch, frozen_flow_sequence
    from synth.kl import kl_modes

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg, B = CFG2, args.batch
    P = cfg.n_pupil

    log("inputs")
    opd_host, r0 = open_loop_batch(cfg, ATMO2, list(range(args.seed, args.seed + B)), r0_range=CFG4_R0_RANGE)
    opd = torch.from_numpy(opd_host).to(dev)
    plan = pw.Plan(cfg, batch_max=B)
    nv = plan.n_valid
    ns = 2 * nv

    # Calibration: KL modal DM, push-pull interaction matrix measured on the
    # GPU, full-SVD pseudo-inverse on the host (FP64).
    log("calibration")
    t0 = time.time()
    amp = plan.pupil.astype(np.float64)
    s_buf = torch.empty((B, ns), device=dev)
    if args.random_R:
        args.no_loop = True
        args.no_cnn = True
        args.no_multi = True
        M = N_KL_MODES
        R_host = np.random.default_rng(0).standard_normal((M, ns)) * 1e-2
    else:
        modes = kl_modes(amp, cfg.pixel_m, ATMO2.L0_m, N_KL_MODES)
        M = modes.shape[0]
        modes_dev = torch.from_numpy(modes.astype(np.float32)).to(dev)
        if args.calib_dir:
            from paper_1607_07624_amd.calib import CalibrationStore, calibrate_cached
            R, _, sig, hit = calibrate_cached(plan, modes.astype(np.float32), PUSH_PULL_NM,
                                              CalibrationStore(args.calib_dir), device=dev)
            log(f"calibration cache {'hit' if hit else 'miss (measured and stored)'} in {args.calib_dir}")
        else:
            R, _, sig = calibrate(plan, modes.astype(np.float32), PUSH_PULL_NM, dev)
        log(f"IM condition number {sig[0] / sig[-1]:.1f}")
    if args.random_R:
        R = torch.from_numpy(R_host.astype(np.float32)).to(dev).contiguous()
    log(f"calibration {time.time() - t0:.1f}s")

    modes_out = torch.empty((B, M), device=dev)

    def step():
        plan.measure_into(opd, None, s_buf)
        pw.recon_apply(R, s_buf, 1.0, 0.0, modes_out)

    # Work split chosen by the library's autotuner (set-up, outside the timed region).
    schedule = {"B": B, "a_chunk": None, "k_chunk": None, "autotuned": False}
    schedule["a_chunk"], schedule["k_chunk"] = plan.get_schedule(B)
    if args.schedule:
        a_k = [int(v) for v in args.schedule.split(",")]
        plan.set_schedule(B, a_k[0], a_k[1])
        schedule["a_chunk"], schedule["k_chunk"] = plan.get_schedule(B)
    elif not args.no_autotune:
        schedule = plan.autotune(B, reps=5)
        schedule["autotuned"] = True
        log(f"autotune {schedule}")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps
    fps = B * args.steps / (ms_total / 1e3)
    # Kernel durations: the same K steps again with the library's events bound
    # to its kernels (their start and end times).  Timed kernels cost the
    # stream ~20 us per step, so the throughput above is taken without them.
    plan.timing_enable(True)
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    ms_step_timed = ev0.elapsed_time(ev1) / args.steps
    kt = plan.timing_read()
    plan.timing_enable(False)
    # recon_apply alone, K calls on the step's slopes
    ev0.record()
    for _ in range(args.steps):
        pw.recon_apply(R, s_buf, 1.0, 0.0, modes_out)
    ev1.record()
    torch.cuda.synchronize()
    recon_ms = ev0.elapsed_time(ev1) / args.steps
    log(f"{fps:.0f} frames/s, {ms_step:.3f} ms/step (wall {wall:.2f}s; with kernel timing {ms_step_timed:.3f} ms/step)"
        f" kernels {kt}")
    repeats = median_of_repeats(step, max(1, args.repeat_frames // B), B, ev0, ev1) if args.repeat_frames > 0 else None
    log(f"repeats {repeats}")

    if args.copy_mb:
        n = args.copy_mb * (1 << 20) // 4
        src = torch.ones(n, device=dev)
        dst = torch.empty(n, device=dev)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy of {args.copy_mb} MiB done")
        del src, dst

    # Roofline of the column pass (dominant kernel).
    n_launch = kt["slices"]
    col_ms = kt["col_ms"] / n_launch
    row_ms = kt["row_ms"] / n_launch
    lines_col = B * cfg.n_mod * 2 * P
    lines_row = B * (cfg.n_mod // 2 + 1) * P
    fl_col = lines_col * line_flops(P, True)
    fl_row = lines_row * line_flops(P, False)
    # Algorithmic work: two N-point FFTs per column line at 5 N log2 N flops
    # each (the transform count of the separable schedule); the issued count of
    # the reduced line operator (`line_flops`) is reported beside it.
    conv = lines_col * fft_pair_flops(cfg.n_fft)
    achieved = conv / (col_ms * 1e-3) / 1e12
    issued = fl_col / (col_ms * 1e-3) / 1e12
    traffic = counter_traffic(B, (schedule["a_chunk"], schedule["k_chunk"]))
    roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": traffic, "traffic_unit": "bytes per launch (rocprofv3 counters)",
                "hbm_frac_of_peak": (round(traffic / (col_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
                                     if traffic else None),
                "kernel": "col_pass_kernel<40, 4>", "kernel_ms": round(col_ms, 4),
                "flop_per_launch": int(conv), "flop_convention": "2 x 5 N log2 N per column line, N = 640",
                "issued_flop_per_launch": int(fl_col), "issued_tflops": round(issued, 2),
                "issued_frac": round(issued / PEAK_FP32_TFLOPS, 4)}
    extra = {"row_pass_ms": round(row_ms, 4),
             "row_pass_tflops": round(lines_row * fft_pair_flops(cfg.n_fft) / (row_ms * 1e-3) / 1e12, 2),
             "row_pass_issued_tflops": round(fl_row / (row_ms * 1e-3) / 1e12, 2),
             "slopes_ms": round(kt["slopes_ms"] / n_launch, 4),
             "recon_ms": round(recon_ms, 4),
             "timing": ("kernel durations from events bound to the kernels' start and end "
                        "(hipExtLaunchKernel) over a second pass of the same K steps; "
                        f"that pass ran at {ms_step_timed:.4f} ms/step")}

    # B = 1 latency (one frame per call, same path).
    plan1 = pw.Plan(cfg, batch_max=1)
    if not args.no_autotune and not args.schedule:
        extra["b1_schedule"] = plan1.autotune(1, reps=5)
        log(f"autotune B=1 {extra['b1_schedule']}")
    s1 = torch.empty((1, ns), device=dev)
    m1 = torch.empty((1, M), device=dev)
    o1 = opd[:1].contiguous()
    for _ in range(20):
        plan1.measure_into(o1, None, s1)
        pw.recon_apply(R, s1, 1.0, 0.0, m1)
    torch.cuda.synchronize()
    ev0.record()
    n1 = 200
    for _ in range(n1):
        plan1.measure_into(o1, None, s1)
        pw.recon_apply(R, s1, 1.0, 0.0, m1)
    ev1.record()
    torch.cuda.synchronize()
    extra["b1_frames_per_s"] = round(n1 / (ev0.elapsed_time(ev1) / 1e3), 1)

    def step1():
        plan1.measure_into(o1, None, s1)
        pw.recon_apply(R, s1, 1.0, 0.0, m1)
    if args.repeat_frames > 0:
        extra["b1_repeats"] = median_of_repeats(step1, args.repeat_frames, 1, ev0, ev1)

    # The paper's detector geometry (80 x 80 frame, pupils 30 px across and 36
    # apart: each P = 160 window rebinned to 36 px), valid list from the pupil
    # acquisition on a flat frame at 20 lambda/D; same batch, same path.
    if not args.random_R:
        from synth.configs import CFG_PAPER_DET, paper_pupil
        from paper_1607_07624_amd.loop import acquire_valid
        pamp = paper_pupil(CFG_PAPER_DET.n_pupil)
        pplan = pw.Plan(CFG_PAPER_DET, batch_max=B, pupil_amp=pamp)
        n_fill = pplan.n_valid
        pplan.set_valid(acquire_valid(CFG_PAPER_DET, pamp))
        if not args.no_autotune and not args.schedule:
            pplan.autotune(B, reps=3)
        popd = torch.from_numpy(open_loop_batch(CFG_PAPER_DET, ATMO2, list(range(B)), r0_range=CFG4_R0_RANGE)[0]).to(dev)
        ps = torch.empty((B, 2 * pplan.n_valid), device=dev)
        for _ in range(5):
            pplan.measure_into(popd, None, ps)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(50):
            pplan.measure_into(popd, None, ps)
        ev1.record()
        torch.cuda.synchronize()
        extra["paper_detector"] = {"geometry": "80 x 80 px, pupils 30 px across 36 apart (160-px windows to 36 px)",
                                   "n_valid_acquired": pplan.n_valid, "n_valid_fill_rule": n_fill,
                                   "frames_per_s": round(B * 50 / (ev0.elapsed_time(ev1) / 1e3), 1)}
        # The same sensor with the paper's 2 arcsec field stop: the general 2-D path.
        fov_lod = 2.0 / (206264.806 * CFG_PAPER_DET.wavelength_m / 8.4) * 36 / 30
        fplan = pw.Plan(CFG_PAPER_DET.with_(field_stop_lod=fov_lod), batch_max=B, pupil_amp=pamp)
        fplan.set_valid(pplan.valid)
        fs_ = torch.empty((B, 2 * fplan.n_valid), device=dev)
        for _ in range(3):
            fplan.measure_into(popd, None, fs_)
        torch.cuda.synchronize()
        fplan.timing_enable(True)
        ev0.record()
        for _ in range(10):
            fplan.measure_into(popd, None, fs_)
        ev1.record()
        torch.cuda.synchronize()
        kt = fplan.timing_read()
        fplan.timing_enable(False)
        extra["paper_detector"]["with_field_stop"] = {
            "fov_lambda_over_d": round(fov_lod * 30 / 36, 1), "frames_per_s": round(B * 10 / (ev0.elapsed_time(ev1) / 1e3), 1),
            "rows_ms": round(kt["row_ms"] / kt["slices"], 4), "columns_and_output_ms": round(kt["col_ms"] / kt["slices"], 4)}
        log(f"paper detector geometry {extra['paper_detector']}")
        fplan.close()
        pplan.close()

    # Closed loop on the GPU (frozen flow, 1 kHz, 15 m/s).
    loop = None
    if not args.no_loop:
        log("closed loop")
        T = args.loop_steps
        seq = torch.from_numpy(frozen_flow_sequence(cfg, ATMO2, T, seed=2024)).to(dev)
        cl = ClosedLoop(plan1, modes_dev, R, LOOP_GAIN, LOOP_DELAY)
        torch.cuda.synchronize()
        ev0.record()
        res_eager, _ = cl.run(seq)
        ev1.record()
        torch.cuda.synchronize()
        eager_ms = ev0.elapsed_time(ev1)
        # The same loop replayed from captured HIP graphs of 50 steps (same
        # residuals bit for bit): the first run includes the capture, the
        # second replays the kept graphs.
        ev0.record()
        res, _ = cl.run_graph(seq)
        ev1.record()
        torch.cuda.synchronize()
        graph_ms = ev0.elapsed_time(ev1)
        graph_same = bool(torch.equal(res, res_eager))
        ev0.record()
        res, _ = cl.run_graph(seq)
        ev1.record()
        torch.cuda.synchronize()
        replay_ms = ev0.elapsed_time(ev1)
        graph_same = graph_same and bool(torch.equal(res, res_eager))
        res, loop_ms = res_eager, eager_ms
        per_step = residual_rms_nm(res.cpu().numpy(), amp)
        ol = residual_rms_nm(seq.cpu().numpy().reshape(T, -1), amp)
        loop = {"steps": T, "residual_nm_rms": round(float(np.sqrt(np.mean(per_step[LOOP_SETTLE_STEPS:] ** 2))), 2),
                "open_loop_nm_rms": round(float(np.sqrt(np.mean(ol[LOOP_SETTLE_STEPS:] ** 2))), 2),
                "steps_per_s": round(T / (loop_ms / 1e3), 1),
                "graph_replay": {"steps_per_graph": 50, "steps_per_s_with_capture": round(T / (graph_ms / 1e3), 1),
                                 "steps_per_s": round(T / (replay_ms / 1e3), 1), "equals_eager": graph_same},
                "gain": LOOP_GAIN, "delay": LOOP_DELAY,
                "reconstructor": "linear (KL 600, push-pull IM, full-SVD pinv)"}
        cam = pw.PsfCamera(P, 8, 1.65e-6, batch_max=B)
        loop.update(strehl_stats(cam, res, P, LOOP_SETTLE_STEPS))
        rr = res.view(T, P, P)[LOOP_SETTLE_STEPS:].contiguous()
        torch.cuda.synchronize()
        ev0.record()
        cam.compute(rr, accumulate=True)
        ev1.record()
        torch.cuda.synchronize()
        loop["psf_camera_frames_per_s"] = round(rr.shape[0] / (ev0.elapsed_time(ev1) / 1e3), 1)
        del rr
        log(f"loop {loop}")
        # Monte-Carlo realisations advanced as one batch (one measure of B frames per step).
        nr = B
        seqs = np.stack([frozen_flow_sequence(cfg, ATMO2, T, seed=3000 + i, screen_n=1024) for i in range(nr)],
                        axis=1)
        seqs = torch.from_numpy(seqs).to(dev)
        bl = BatchedLoop(plan, modes_dev, R, LOOP_GAIN, LOOP_DELAY)
        torch.cuda.synchronize()
        ev0.record()
        resb, _ = bl.run(seqs)
        ev1.record()
        torch.cuda.synchronize()
        bl_ms = ev0.elapsed_time(ev1)
        resb = resb.cpu().numpy()
        per_real = [float(np.sqrt(np.mean(residual_rms_nm(resb[:, i], amp)[LOOP_SETTLE_STEPS:] ** 2)))
                    for i in range(nr)]
        del seqs, resb
        loop["batched"] = {"realisations": nr, "steps": T,
                           "realisation_steps_per_s": round(nr * T / (bl_ms / 1e3), 1),
                           "residual_nm_rms_mean": round(float(np.mean(per_real)), 2),
                           "residual_nm_rms_std": round(float(np.std(per_real)), 2)}
        log(f"batched loops {loop['batched']}")
        # The paper's example detector: magnitude-8 source, 300 nm band, QE 0.32, 1 e- readout noise.
        from synth.configs import photoelectrons_per_frame, DETECTOR_RON_E
        e_frame = photoelectrons_per_frame(cfg)
        plan1.set_detector(e_frame, DETECTOR_RON_E, seed=8)
        cl = ClosedLoop(plan1, modes_dev, R, LOOP_GAIN, LOOP_DELAY)
        torch.cuda.synchronize()
        ev0.record()
        resn, _ = cl.run(seq)
        ev1.record()
        torch.cuda.synchronize()
        per_step = residual_rms_nm(resn.cpu().numpy(), amp)
        loop["with_detector"] = {"electrons_per_frame": round(e_frame, 1), "readout_noise_e": DETECTOR_RON_E,
                                 "residual_nm_rms": round(float(np.sqrt(np.mean(per_step[LOOP_SETTLE_STEPS:] ** 2))), 2),
                                 "steps_per_s": round(T / (ev0.elapsed_time(ev1) / 1e3), 1)}
        plan1.set_detector(0.0)
        del resn
        log(f"loop with detector {loop['with_detector']}")
        # The same loop sensed by a Shack-Hartmann (40 x 40 subapertures of 4 px, spots padded x4).
        shb = pw.ShPlan(P, 40, 4, cfg.wavelength_m, batch_max=B)
        R_sh, _, _ = calibrate(shb, modes.astype(np.float32), PUSH_PULL_NM, dev)
        sh1 = pw.ShPlan(P, 40, 4, cfg.wavelength_m, batch_max=1)
        cl = ClosedLoop(sh1, modes_dev, R_sh, LOOP_GAIN, LOOP_DELAY)
        torch.cuda.synchronize()
        ev0.record()
        ress, _ = cl.run(seq)
        ev1.record()
        torch.cuda.synchronize()
        per_step = residual_rms_nm(ress.cpu().numpy(), amp)
        loop["shack_hartmann"] = {"sensor": "40 x 40 subapertures of 4 px, spots padded x4, centre of gravity",
                                  "residual_nm_rms": round(float(np.sqrt(np.mean(per_step[LOOP_SETTLE_STEPS:] ** 2))), 2),
                                  "steps_per_s": round(T / (ev0.elapsed_time(ev1) / 1e3), 1)}
        loop["shack_hartmann"].update(strehl_stats(cam, ress, P, LOOP_SETTLE_STEPS))
        del ress
        shb.close()
        sh1.close()
        log(f"Shack-Hartmann loop {loop['shack_hartmann']}")
        plan.set_detector(e_frame, DETECTOR_RON_E, seed=9)
        for _ in range(5):
            step()
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(50):
            step()
        ev1.record()
        torch.cuda.synchronize()
        plan.set_detector(0.0)
        extra["with_detector_frames_per_s"] = round(B * 50 / (ev0.elapsed_time(ev1) / 1e3), 1)

    # Learned reconstructor: trained on GPU-generated frames with the project's
    # kernels, compared with the linear one (held-out open-loop error, closed loop).
    learned = None
    if not args.no_cnn:
        from synth.screens import CropBank
        from synth.configs import AtmoConfig
        from paper_1607_07624_amd.learned import train_reconstructor, open_loop_errors, ResidualBank
        log("learned reconstructor: data + training")
        T = args.loop_steps
        bank = CropBank(cfg, ATMO2.L0_m, n_screens=4, screen_n=4096, seed=4242)
        t_res = time.time()
        resid = ResidualBank.from_loops(plan1, modes_dev, R, cfg, ATMO2.L0_m, ATMO2.wind_m_s, ATMO2.frame_rate_hz,
                                        n_loops=12, steps=1500, settle=LOOP_SETTLE_STEPS, seed=77,
                                        r0_range=(0.06, 0.2), gain=LOOP_GAIN, delay=LOOP_DELAY, stride=2)
        log(f"residual bank {tuple(resid.frames.shape)} in {time.time() - t_res:.1f}s")
        net, info = train_reconstructor(plan, R, modes.astype(np.float32), amp, bank, args.cnn_frames, seed=5,
                                        epochs=args.cnn_epochs, residuals=resid, log=log)
        info["residual_bank_frames"] = int(resid.frames.shape[0])
        del resid
        log(f"training {info}")
        ev_strong = open_loop_errors(plan, net, R, modes.astype(np.float32), amp, bank, 2048, seed=990,
                                     r0_range=(0.06, 0.1))
        ev_all = open_loop_errors(plan, net, R, modes.astype(np.float32), amp, bank, 2048, seed=991,
                                  r0_range=(0.06, 0.2))
        loops = {}
        cam_h = pw.PsfCamera(P, 8, 1.65e-6, batch_max=16)
        for r0 in (0.12, 0.08):
            atm = AtmoConfig(r0_m=r0, L0_m=ATMO2.L0_m, wind_m_s=ATMO2.wind_m_s, frame_rate_hz=ATMO2.frame_rate_hz)
            sq = torch.from_numpy(frozen_flow_sequence(cfg, atm, T, seed=2024)).to(dev)
            row = {}
            for name, nn_ in (("linear", None), ("cnn", net)):
                cl = ClosedLoop(plan1, modes_dev, R, LOOP_GAIN, LOOP_DELAY, net=nn_)
                torch.cuda.synchronize()
                ev0.record()
                rs, _ = cl.run(sq)
                ev1.record()
                torch.cuda.synchronize()
                ps = residual_rms_nm(rs.cpu().numpy(), amp)
                row[name] = {"residual_nm_rms": round(float(np.sqrt(np.mean(ps[LOOP_SETTLE_STEPS:] ** 2))), 2),
                             "steps_per_s": round(T / (ev0.elapsed_time(ev1) / 1e3), 1)}
                row[name].update(strehl_stats(cam_h, rs, P, LOOP_SETTLE_STEPS))
                if nn_ is not None:
                    row[name]["fallback_step"] = cl.fallback_step
                    g = [v for (tt, v) in cl.judged if tt >= cl.judge_settle]
                    row[name]["optical_gain_mean"] = round(float(np.mean(g)), 3) if g else None
            loops[f"r0_{r0}"] = row
            log(f"loop r0={r0}: {row}")
        # The network's kernels alone on random data: a training step at batch
        # 256 and the forward at 1 and 16 frames, with their bf16 flop rates.
        from paper_1607_07624_amd.cnn_timing import measure as cnn_kernel_rates
        kr = cnn_kernel_rates(batch=256, steps=50)
        kr["train"]["frac_of_bf16_peak"] = round(kr["train"]["tflops"] / kr["peak_bf16_tflops"], 5)
        log(f"cnn kernels {kr}")
        learned = {"training": {k: v for k, v in info.items() if k != "loss_history"},
                   "loss_first_last": [round(info["loss_history"][0], 4), round(info["loss_history"][-1], 4)],
                   "open_loop_error_r0_0.06_0.1": ev_strong, "open_loop_error_r0_0.06_0.2": ev_all,
                   "closed_loop": loops, "kernels": kr}

    multi = None
    if not args.no_multi:
        multi = multi_source_leg(args, log)

    # CPU baseline: the FP64 oracle on the host cores, small sample.
    cpu = None
    if not args.no_cpu:
        cores = len(os.sched_getaffinity(0))
        import oracle
        import oracle.pwfs as opw
        orc = oracle.Oracle(cfg)
        n = min(args.cpu_frames, B)
        opw._WORKERS = cores
        t0 = time.perf_counter()
        for i in range(n):
            orc.measure(opd_host[i].astype(np.float64))
        dt = time.perf_counter() - t0
        n1c = min(args.cpu_frames_1core, B)
        opw._WORKERS = 1
        t0 = time.perf_counter()
        for i in range(n1c):
            orc.measure(opd_host[i].astype(np.float64))
        dt1 = time.perf_counter() - t0
        cpu = {"value": round(n / dt, 4), "unit": "frames/s", "cores": cores, "kind": "oracle",
               "sample": f"{n} of the {B} benchmark frames, FP64 literal 2-D route, scipy.fft workers={cores}",
               "value_1core": round(n1c / dt1, 4),
               "sample_1core": f"{n1c} of the same frames, scipy.fft workers=1",
               "cpu_model": cpu_model()}
        log(f"cpu {cpu}")

    out = {
        "metric": "PWFS frames/s at 640^2 FFT, 48 mod pts",
        "value": round(fps, 1), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "lbt_like_pwfs_n640_p160_k48_s40_b16", "frames_per_step": B,
                   "n_fft": cfg.n_fft, "n_pupil": P, "n_mod": cfg.n_mod, "n_sub": cfg.n_sub,
                   "n_valid": nv, "n_modes": M, "screens": "von Karman r0~U[0.08,0.2] m, L0=40 m",
                   "step": "pwfs_measure + recon_apply"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "timing_protocol": repeats,
        "loop": loop,
        "learned": learned,
        "multi_source": multi,
        "kernels": extra,
        "schedule": schedule,
    }
    print(json.dumps(out), flush=True)
    if args.jsonl:
        with open(args.jsonl, "a") as f:
            f.write(json.dumps(dict(out, argv=sys.argv[1:], unix_time=round(time.time(), 1))) + "\n")


if __name__ == "__main__":
    main()
