"""The paper's detector geometry through the C ABI: each pupil window
resampled to the detector's pixels (output resolution 80, pupils 30 pixels
across, 36 apart: a non-integer rebin of P = 160 windows to 36 pixels), its
pupil acquisition on a flat frame with a 20 lambda/D modulation, and the
replacement of the valid list.  Gates as in test_gpu_pwfs."""
import numpy as np
import pytest

from synth.configs import CFG_PAPER_DET, ATMO1, ATMO2, SensorConfig, paper_pupil
from synth.screens import open_loop_batch
import oracle
from tests.gpu_common import torch_cuda, rel_l2, say, check_frame

pytestmark = pytest.mark.gpu

SLOPE_TOL = 1e-5
PUPIL_TOL = 2e-6

CFG_SMALL = SensorConfig(name="p32_det7_k12_obs_norm1", n_fft=128, n_pupil=32, n_bin=1, n_mod=12,
                         mod_radius_lod=2.5, wavelength_m=750e-9, diameter_m=8.0, obstruction=0.2,
                         norm_mode=1, det_window=7)
CFG_ACQ = SensorConfig(name="p64_det14_k24", n_fft=256, n_pupil=64, n_bin=1, n_mod=24, mod_radius_lod=3.6,
                       wavelength_m=750e-9, diameter_m=9.6, det_window=14)


def _check(cfg, A, opd, batch_max, plan=None, orc=None):
    import paper_1607_07624_amd as pw
    torch = torch_cuda()
    own = plan is None
    plan = plan or pw.Plan(cfg, batch_max=batch_max, pupil_amp=A)
    orc = orc or oracle.Oracle(cfg, None if A is None else A.astype(np.float64))
    assert plan.n_sub == cfg.det_window
    assert np.array_equal(plan.valid, orc.valid)
    e = float(np.abs(plan.s_ref.astype(np.float64) - orc.s_ref).max())
    say(f"[gpu] {cfg.name}: {plan.n_valid} valid, reference slope max abs err {e:.3e}")
    assert e <= 1e-6
    pup, s = plan.measure(torch.from_numpy(np.ascontiguousarray(opd)).cuda())
    torch.cuda.synchronize()
    pup, s = pup.cpu().numpy(), s.cpu().numpy()
    for i in range(len(opd)):
        p_o, s_o = orc.measure(opd[i].astype(np.float64))
        check_frame(f"frame {i}", s[i], s_o, pup[i], p_o)
    if own:
        plan.close()


def test_paper_detector_geometry():
    """P = 160 windows to 36 detector pixels (pitch 40/9), pupil 133.3 pixels across."""
    A = paper_pupil(160)
    opd, _ = open_loop_batch(CFG_PAPER_DET, ATMO2, [60, 61])
    _check(CFG_PAPER_DET, A, opd, batch_max=2)


def test_non_integer_rebin_small_ragged():
    """P = 32 to 7 pixels (pitch 32/7), obstruction, per-subaperture
    normalisation, three frames in slices of two."""
    opd, _ = open_loop_batch(CFG_SMALL, ATMO1, [62, 63, 64], screen_n=64)
    _check(CFG_SMALL, None, opd, batch_max=2)


def test_rebinned_images_through_the_detector():
    """With a detector set, the rebinned noiseless images go through the same
    counter-based noise as pwfs_detect applied to them afterwards."""
    import paper_1607_07624_amd as pw
    torch = torch_cuda()
    plan = pw.Plan(CFG_SMALL, batch_max=3)
    opd, _ = open_loop_batch(CFG_SMALL, ATMO1, [65, 66, 67], screen_n=64)
    d = torch.from_numpy(np.ascontiguousarray(opd)).cuda()
    clean, _ = plan.measure(d)
    plan.set_detector(5.0e4, 1.0, seed=11)
    pix, _ = plan.measure(d)
    again = plan.detect(clean, frame0=0)
    torch.cuda.synchronize()
    assert torch.equal(pix, again)
    g = plan.detector()["gain"]
    assert abs(float(pix.sum()) / (g * float(clean.sum())) - 1.0) < 0.01
    plan.close()


def test_acquisition_and_replaced_valid_list():
    import paper_1607_07624_amd as pw
    from paper_1607_07624_amd._lib import PwfsError
    from paper_1607_07624_amd.loop import acquire_valid
    torch = torch_cuda()
    A = paper_pupil(64)
    thr = 0.5
    idx = acquire_valid(CFG_ACQ, A, thr=thr, mod_radius_lod=20.0, n_mod=128)
    acq_cfg = CFG_ACQ.with_(mod_radius_lod=20.0, n_mod=128)
    pup_o = oracle.pupil_images(acq_cfg, oracle.intensity(acq_cfg, np.zeros((64, 64)), A.astype(np.float64)))
    idx_o = oracle.acquire_valid(pup_o, thr)
    tot = pup_o.sum(axis=0).ravel() / pup_o.sum(axis=0).max()
    diff = sorted(set(idx.tolist()) ^ set(idx_o.tolist()))
    say(f"[gpu] acquisition: {idx.size} subapertures (oracle {idx_o.size}), {len(diff)} differ")
    assert all(abs(tot[j] - thr) < 1e-5 for j in diff)
    plan = pw.Plan(CFG_ACQ, batch_max=2, pupil_amp=A)
    before = plan.valid.copy()
    for bad in (idx[::-1], np.array([], np.int32), np.array([0, 14 * 14], np.int32), np.array([3, 3], np.int32)):
        with pytest.raises(PwfsError):
            plan.set_valid(bad)
    assert np.array_equal(plan.valid, before)
    plan.set_valid(idx)
    assert plan.n_valid == idx.size and np.array_equal(plan.valid, idx)
    orc = oracle.Oracle(CFG_ACQ, A.astype(np.float64), valid=idx)
    opd, _ = open_loop_batch(CFG_ACQ, ATMO2, [68, 69], screen_n=256)
    _check(CFG_ACQ.with_(name="p64_det14_acquired"), A, opd, batch_max=2, plan=plan, orc=orc)
    plan.close()
