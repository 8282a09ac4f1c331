"""Shack-Hartmann sensor through the C ABI against the FP64 reference in
oracle/sh.py: spots, reference centroids and slopes (relative L2 <= 1e-5,
FP32 direct DFT and moment sums), and a closed loop driven by it against the
oracle's loop (same tolerances as the pyramid loop)."""
import numpy as np
import pytest

from synth.configs import CFG1, CFG2, ATMO1, ATMO2, AtmoConfig, PUSH_PULL_NM, LOOP_GAIN, LOOP_DELAY, \
    LOOP_SETTLE_STEPS
from synth.screens import open_loop_batch, frozen_flow_sequence
from synth.kl import kl_modes
import oracle
from oracle import recon as orecon
from oracle.sh import ShackHartmann
from tests.gpu_common import torch_cuda, rel_l2, say

pytestmark = pytest.mark.gpu


def _check(P, n_sub, pad, lam, opd, batch_max):
    import paper_1607_07624_amd as pw
    torch = torch_cuda()
    sh = pw.ShPlan(P, n_sub, pad, lam, batch_max=batch_max)
    ref = ShackHartmann(P, n_sub, pad, lam)
    assert np.array_equal(sh.valid, ref.valid)
    e_ref = float(np.abs(sh.s_ref - ref.ref).max())
    spots, s = sh.measure(torch.from_numpy(np.ascontiguousarray(opd)).cuda())
    spots, s = spots.cpu().numpy(), s.cpu().numpy()
    worst = 0.0
    for i in range(len(opd)):
        sp_o, s_o = ref.measure(opd[i].astype(np.float64))
        e_s, e_p = rel_l2(s[i], s_o), rel_l2(spots[i], sp_o)
        worst = max(worst, e_s)
        assert e_s <= 1e-5 and e_p <= 1e-5, (i, e_s, e_p)
    say(f"[gpu] SH P={P} n_sub={n_sub} pad={pad}: {sh.n_valid} valid, reference max abs err {e_ref:.2e} px, "
        f"worst slope rel err {worst:.3e}")
    assert e_ref <= 1e-5
    return sh


def test_sh_small_geometry():
    opd, _ = open_loop_batch(CFG1, ATMO1, [80, 81, 82, 83, 84], screen_n=64)
    _check(32, 8, 4, 750e-9, 0.3 * opd, batch_max=2).close()        # slices of 2, ragged tail
    _check(32, 16, 2, 750e-9, 0.3 * opd[:2], batch_max=2).close()   # 2-pixel subapertures


def test_sh_lbt_like_geometry():
    opd, _ = open_loop_batch(CFG2, ATMO2, [85, 86])
    _check(160, 40, 4, 750e-9, 0.3 * opd, batch_max=2).close()


def test_sh_closed_loop_matches_oracle():
    import paper_1607_07624_amd as pw
    from paper_1607_07624_amd.loop import calibrate, ClosedLoop, residual_rms_nm
    torch = torch_cuda()
    T = 150
    A = oracle.pupil_amplitude(32, 0.0)
    modes = kl_modes(A, CFG1.pixel_m, 25.0, 40).astype(np.float32)
    seq = frozen_flow_sequence(CFG1, AtmoConfig(r0_m=0.5, L0_m=25.0, wind_m_s=15.0), T, seed=9, screen_n=256)
    R_g, _, _ = calibrate(pw.ShPlan(32, 8, 4, 750e-9, batch_max=16), modes, PUSH_PULL_NM)
    sh1 = pw.ShPlan(32, 8, 4, 750e-9, batch_max=1)
    res, _ = ClosedLoop(sh1, torch.from_numpy(modes).cuda(), R_g, LOOP_GAIN, LOOP_DELAY).run(
        torch.from_numpy(seq).cuda())
    rms_g = residual_rms_nm(res.cpu().numpy(), A)
    ref = ShackHartmann(32, 8, 4, 750e-9)
    meas = lambda r: ref.measure(r)[1]
    IM_o = orecon.interaction_matrix(meas, modes.astype(np.float64), PUSH_PULL_NM)
    R_o, _ = orecon.pseudo_inverse(IM_o)
    rms_o, _ = orecon.closed_loop(meas, seq, modes.astype(np.float64), R_o, LOOP_GAIN, LOOP_DELAY, A)
    tot_g = orecon.loop_residual_nm(rms_g, LOOP_SETTLE_STEPS)
    tot_o = orecon.loop_residual_nm(rms_o, LOOP_SETTLE_STEPS)
    ol = orecon.loop_residual_nm(residual_rms_nm(seq.reshape(T, -1), A), LOOP_SETTLE_STEPS)
    worst = float(np.max(np.abs(rms_g - rms_o) / rms_o))
    say(f"[gpu] SH loop: residual {tot_g:.4f} nm (oracle {tot_o:.4f} nm, open loop {ol:.1f} nm), "
        f"worst per-step rel diff {worst:.3e}")
    assert tot_o < 0.5 * ol
    assert worst <= 1e-3
    assert abs(tot_g - tot_o) <= 1e-4 * tot_o
