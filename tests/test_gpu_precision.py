"""Precision study on the LBT-like shapes: FP64-generated tables and FP64
phase formation (default) against FP32-generated tables and/or FP32 phase,
slopes compared with the FP64 oracle on 16 seeded screens
(r0 ~ U[0.08, 0.2] m), plus the 500-step closed-loop residual of each
setting.  The default is gated at the 1e-5 slope bound; the FP32 variants
are reported and only required to stay below 1e-3."""
import numpy as np
import pytest

from synth.configs import CFG2, ATMO2, CFG4_R0_RANGE, CFG4_SEEDS, PUSH_PULL_NM, LOOP_GAIN, LOOP_DELAY, \
    LOOP_SETTLE_STEPS
from synth.screens import open_loop_batch, frozen_flow_sequence
from synth.kl import kl_modes
import oracle
from tests.gpu_common import torch_cuda, rel_l2, say

pytestmark = pytest.mark.gpu

SETTINGS = {"fp64_tables_fp64_phase": 0, "fp32_tables": 1, "fp32_phase": 2, "fp32_tables_fp32_phase": 3}


def test_precision_study_slopes_and_loop():
    import paper_1607_07624_amd as pw
    from paper_1607_07624_amd.loop import calibrate, ClosedLoop, residual_rms_nm
    torch = torch_cuda()
    opd, r0 = open_loop_batch(CFG2, ATMO2, list(CFG4_SEEDS), r0_range=CFG4_R0_RANGE)
    orc = oracle.Oracle(CFG2)
    s_orc = np.stack([orc.measure(o.astype(np.float64))[1] for o in opd])
    d_opd = torch.from_numpy(opd).cuda()
    pupil = None
    modes = None
    seq = torch.from_numpy(frozen_flow_sequence(CFG2, ATMO2, 500, seed=4)).cuda()
    results = {}
    for name, flags in SETTINGS.items():
        plan = pw.Plan(CFG2, batch_max=16, flags=flags)
        _, s = plan.measure(d_opd, want_pupils=False)
        s = s.cpu().numpy()
        errs = np.array([rel_l2(s[i], s_orc[i]) for i in range(len(opd))])
        if modes is None:
            pupil = plan.pupil.astype(np.float64)
            modes = kl_modes(pupil, CFG2.pixel_m, ATMO2.L0_m, 600).astype(np.float32)
        R, _, _ = calibrate(plan, modes, PUSH_PULL_NM)
        plan1 = pw.Plan(CFG2, batch_max=1, flags=flags)
        res, _ = ClosedLoop(plan1, torch.from_numpy(modes).cuda(), R, LOOP_GAIN, LOOP_DELAY).run(seq)
        rms = residual_rms_nm(res.cpu().numpy(), pupil)
        tot = float(np.sqrt(np.mean(rms[LOOP_SETTLE_STEPS:] ** 2)))
        results[name] = (errs, tot)
        say(f"[gpu] precision {name}: slope rel err max {errs.max():.3e} median {np.median(errs):.3e} "
            f"per frame {np.array2string(errs, precision=2, max_line_width=400)}; loop residual {tot:.4f} nm")
    base = results["fp64_tables_fp64_phase"]
    assert base[0].max() <= 1e-5
    for name, (errs, tot) in results.items():
        assert errs.max() <= 1e-3, name
        say(f"[gpu] precision {name}: loop residual difference vs default {tot - base[1]:+.4f} nm")
