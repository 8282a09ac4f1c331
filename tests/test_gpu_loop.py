"""Calibration (interaction matrix) and closed loop on the GPU against the oracle.

The GPU side calibrates with its own measurements (push-pull through
pwfs_measure, FP64 pseudo-inverse on the host) and runs the loop through the
C ABI; the oracle side calibrates and runs with the FP64 oracle.  Both use
the same seeded inputs and the same KL modes (FP32-rounded).

Tolerances.  A 10 nm poke moves the intensities by ~1e-2 of their O(1)
values, so FP32 slope differences lose ~2 digits to cancellation: IM
columns are gated at 1e-4 relative.  The loop residual follows the
reconstructor error (~1e-5 relative) through a stable loop: per-step
residual RMS within 1e-3 relative, overall residual within 1e-4.
"""
import numpy as np
import pytest

from synth.configs import CFG1, CFG2, ATMO2, AtmoConfig, PUSH_PULL_NM, LOOP_GAIN, LOOP_DELAY, LOOP_SETTLE_STEPS
from synth.screens import frozen_flow_sequence
from synth.kl import kl_modes
import oracle
from oracle import recon as orecon
from tests.gpu_common import torch_cuda, rel_l2, rel_max, say
from tests import loop_golden

pytestmark = pytest.mark.gpu


def _modes(cfg, L0, M):
    A = oracle.pupil_amplitude(cfg.n_pupil, cfg.obstruction)
    return kl_modes(A, cfg.pixel_m, L0, M).astype(np.float32), A


def test_interaction_matrix_columns_cfg1():
    import paper_1607_07624_amd as pw
    from paper_1607_07624_amd.loop import interaction_matrix
    torch_cuda()
    modes, A = _modes(CFG1, 25.0, 60)
    plan = pw.Plan(CFG1, batch_max=16)
    IM_g = interaction_matrix(plan, modes, PUSH_PULL_NM)
    orc = oracle.Oracle(CFG1)
    IM_o = orecon.interaction_matrix(lambda r: orc.measure(r)[1], modes.astype(np.float64), PUSH_PULL_NM)
    errs = [rel_l2(IM_g[:, i], IM_o[:, i]) for i in range(IM_o.shape[1])]
    say(f"[gpu] IM cfg1: worst column rel err {max(errs):.3e}, median {np.median(errs):.3e}")
    assert max(errs) <= 1e-4


def test_interaction_matrix_all_columns_cfg2():
    """All 600 push-pull columns at the LBT-like shapes against the oracle's
    (stored FP32-rounded, 6e-8 relative), per column in relative L2 and per
    element (max |error| / max |column|), gate 1e-4 as above."""
    import paper_1607_07624_amd as pw
    from paper_1607_07624_amd.loop import interaction_matrix
    torch_cuda()
    IM_o, rec = loop_golden.load()
    modes, A = loop_golden.modes_checked(rec)
    plan = pw.Plan(CFG2, batch_max=16)
    assert np.array_equal(plan.pupil, A) and IM_o.shape == (2 * plan.n_valid, modes.shape[0])
    IM_g = interaction_matrix(plan, modes, PUSH_PULL_NM)
    plan.close()
    errs = np.array([rel_l2(IM_g[:, i], IM_o[:, i]) for i in range(IM_o.shape[1])])
    emax = np.array([rel_max(IM_g[:, i], IM_o[:, i]) for i in range(IM_o.shape[1])])
    say(f"[gpu] IM cfg2, 600 columns: rel err worst {errs.max():.3e} (mode {int(errs.argmax())}), "
        f"median {np.median(errs):.3e}; per element worst {emax.max():.3e}")
    assert errs.max() <= 1e-4 and emax.max() <= 1e-4


def _lbt_loop_case(name):
    """(stored oracle loop record, sequence, modes, pupil, shared FP32 R on the device)."""
    from paper_1607_07624_amd.loop import pseudo_inverse
    torch = torch_cuda()
    IM_o, rec = loop_golden.load()
    modes, A = loop_golden.modes_checked(rec)
    R, _ = pseudo_inverse(IM_o)
    return rec["loops"][name], modes, A, torch.from_numpy(R.astype(np.float32)).cuda().contiguous()


def test_lbt_loop_matches_oracle():
    """The benchmark's loop (r0 0.12 m, 1000 steps of 1 ms, 600 KL modes,
    gain 0.4, delay 2) against the oracle's loop on the same sequence.  Two
    reconstructors: the shared one (pseudo-inverse of the stored oracle IM,
    as the oracle used) and the GPU's own calibration (end to end).  Gates
    as for the small loops: per step 1e-3, residual over t >= 50 1e-4."""
    import paper_1607_07624_amd as pw
    from paper_1607_07624_amd.loop import calibrate, ClosedLoop, residual_rms_nm
    from synth.configs import CFG2_LOOP_SEED, CFG2_LOOP_STEPS
    torch = torch_cuda()
    gold, modes, A, R_shared = _lbt_loop_case(f"cfg2_r0_0.12_seed{CFG2_LOOP_SEED}")
    seq = torch.from_numpy(frozen_flow_sequence(CFG2, ATMO2, CFG2_LOOP_STEPS, seed=CFG2_LOOP_SEED)).cuda()
    plan_cal = pw.Plan(CFG2, batch_max=16)
    R_own, _, _ = calibrate(plan_cal, modes, PUSH_PULL_NM)
    plan_cal.close()
    plan = pw.Plan(CFG2, batch_max=1)
    modes_dev = torch.from_numpy(modes).cuda()
    for label, R in (("shared R", R_shared), ("own calibration", R_own)):
        res, _ = ClosedLoop(plan, modes_dev, R, LOOP_GAIN, LOOP_DELAY).run(seq)
        rms = residual_rms_nm(res.cpu().numpy(), A)
        worst, tot_rel, tg, to = loop_golden.loop_errors(rms, gold["rms_nm"], LOOP_SETTLE_STEPS)
        say(f"[gpu] LBT loop, {label}: residual {tg:.4f} nm (oracle {to:.4f} nm, open loop "
            f"{gold['open_loop_nm']:.1f} nm), worst per-step rel diff {worst:.3e}, residual rel diff {tot_rel:.3e}")
        assert worst <= 1e-3 and tot_rel <= 1e-4, label
    plan.close()


def test_closed_loop_matches_oracle_cfg1():
    import paper_1607_07624_amd as pw
    from paper_1607_07624_amd.loop import calibrate, ClosedLoop, residual_rms_nm, pseudo_inverse
    torch = torch_cuda()
    T = 300
    modes, A = _modes(CFG1, 25.0, 60)
    # r0 = 0.5 m keeps the 8 m, 32-pixel sensor in its linear range, so the
    # 60-mode loop has something to correct (at r0 = 0.15 m the pupil is
    # under-sampled and the sensor saturates).
    atmo = AtmoConfig(r0_m=0.5, L0_m=25.0, wind_m_s=15.0)
    seq = frozen_flow_sequence(CFG1, atmo, T, seed=5, screen_n=256)
    plan_cal = pw.Plan(CFG1, batch_max=16)
    R_g, IM_g, _ = calibrate(plan_cal, modes, PUSH_PULL_NM)
    plan = pw.Plan(CFG1, batch_max=1)
    cl = ClosedLoop(plan, torch.from_numpy(modes).cuda(), R_g, LOOP_GAIN, LOOP_DELAY)
    res, c = cl.run(torch.from_numpy(seq).cuda())
    rms_g = residual_rms_nm(res.cpu().numpy(), A)

    orc = oracle.Oracle(CFG1)
    meas = lambda r: orc.measure(r)[1]
    IM_o = orecon.interaction_matrix(meas, modes.astype(np.float64), PUSH_PULL_NM)
    R_o, _ = orecon.pseudo_inverse(IM_o)
    rms_o, c_o = orecon.closed_loop(meas, seq, modes.astype(np.float64), R_o, LOOP_GAIN, LOOP_DELAY, A)
    tot_g = orecon.loop_residual_nm(rms_g, LOOP_SETTLE_STEPS)
    tot_o = orecon.loop_residual_nm(rms_o, LOOP_SETTLE_STEPS)
    worst = float(np.max(np.abs(rms_g - rms_o) / rms_o))
    ol = residual_rms_nm(seq.reshape(T, -1), A)
    tot_ol = orecon.loop_residual_nm(ol, LOOP_SETTLE_STEPS)
    say(f"[gpu] loop cfg1: residual {tot_g:.4f} nm (oracle {tot_o:.4f} nm), open loop {tot_ol:.1f} nm, "
        f"worst per-step rel diff {worst:.3e}")
    assert tot_o < 0.5 * tot_ol                   # the loop closes
    assert worst <= 1e-3
    assert abs(tot_g - tot_o) <= 1e-4 * tot_o


def test_batched_loops_match_oracle_cfg1():
    """Three Monte-Carlo realisations advanced as one batch: each follows the
    oracle's single closed loop on its own sequence to the tolerances above."""
    import paper_1607_07624_amd as pw
    from paper_1607_07624_amd.loop import calibrate, BatchedLoop, residual_rms_nm
    torch = torch_cuda()
    T, seeds = 150, (11, 12, 13)
    modes, A = _modes(CFG1, 25.0, 60)
    atmo = AtmoConfig(r0_m=0.5, L0_m=25.0, wind_m_s=15.0)
    seqs = np.stack([frozen_flow_sequence(CFG1, atmo, T, seed=sd, screen_n=256) for sd in seeds], axis=1)
    plan_cal = pw.Plan(CFG1, batch_max=16)
    R_g, _, _ = calibrate(plan_cal, modes, PUSH_PULL_NM)
    plan = pw.Plan(CFG1, batch_max=4)
    bl = BatchedLoop(plan, torch.from_numpy(modes).cuda(), R_g, LOOP_GAIN, LOOP_DELAY)
    res, _ = bl.run(torch.from_numpy(np.ascontiguousarray(seqs)).cuda())
    res = res.cpu().numpy()
    orc = oracle.Oracle(CFG1)
    meas = lambda r: orc.measure(r)[1]
    IM_o = orecon.interaction_matrix(meas, modes.astype(np.float64), PUSH_PULL_NM)
    R_o, _ = orecon.pseudo_inverse(IM_o)
    for b, sd in enumerate(seeds):
        rms_g = residual_rms_nm(res[:, b], A)
        rms_o, _ = orecon.closed_loop(meas, seqs[:, b], modes.astype(np.float64), R_o, LOOP_GAIN, LOOP_DELAY, A)
        tot_g = orecon.loop_residual_nm(rms_g, LOOP_SETTLE_STEPS)
        tot_o = orecon.loop_residual_nm(rms_o, LOOP_SETTLE_STEPS)
        worst = float(np.max(np.abs(rms_g - rms_o) / rms_o))
        say(f"[gpu] batched loop cfg1 seed {sd}: residual {tot_g:.4f} nm (oracle {tot_o:.4f} nm), "
            f"worst per-step rel diff {worst:.3e}")
        assert worst <= 1e-3
        assert abs(tot_g - tot_o) <= 1e-4 * tot_o


def test_graph_replayed_loop_equals_eager():
    """The linear loop replayed from captured HIP graphs of L steps each gives
    the eager loop's residuals and commands bit for bit: 120 steps with
    L = 50 (two windows and a 20-step tail graph), 7 (a 1-step tail) and 1
    (one step per graph), delays 2 and 3, each graph replayed several times
    with the loop's own copies between the replays and eager work and
    synchronisations between the runs; a sensor with a detector is refused
    (its frame counter would be frozen)."""
    import paper_1607_07624_amd as pw
    from paper_1607_07624_amd.loop import calibrate, ClosedLoop
    torch = torch_cuda()
    T = 120
    modes, A = _modes(CFG1, 25.0, 60)
    atmo = AtmoConfig(r0_m=0.5, L0_m=25.0, wind_m_s=15.0)
    plan_cal = pw.Plan(CFG1, batch_max=16)
    R_g, _, _ = calibrate(plan_cal, modes, PUSH_PULL_NM)
    plan = pw.Plan(CFG1, batch_max=1)
    modes_dev = torch.from_numpy(modes).cuda()
    for delay, seed, L in ((LOOP_DELAY, 11, 50), (3, 12, 7), (LOOP_DELAY, 13, 1)):
        seq = torch.from_numpy(frozen_flow_sequence(CFG1, atmo, T, seed=seed, screen_n=256)).cuda()
        cl = ClosedLoop(plan, modes_dev, R_g, LOOP_GAIN, delay)
        res_e, c_e = cl.run(seq)
        torch.cuda.synchronize()
        junk = torch.randn(1 << 16, device="cuda").sum()         # eager work between the runs
        res_g, c_g = cl.run_graph(seq, steps_per_graph=L)
        torch.cuda.synchronize()
        say(f"[gpu] graph loop, delay {delay}, {L} steps per graph: residual equal {torch.equal(res_g, res_e)}, "
            f"commands equal {torch.equal(c_g, c_e)} ({float(junk):.1f})")
        assert torch.equal(res_g, res_e) and torch.equal(c_g, c_e)
    plan.set_detector(1.0e5, 1.0, seed=3)
    with pytest.raises(ValueError):
        ClosedLoop(plan, modes_dev, R_g, LOOP_GAIN, LOOP_DELAY).run_graph(seq)
    plan.close()
