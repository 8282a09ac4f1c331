"""pwfs_measure_static (no allocation: the workspace comes from the library's
static device array) against pwfs_measure on the same plan and inputs.

Both entry points run the same slices, schedules and kernels, so the
images and slopes must agree bit for bit; each case makes two calls in a
row, the second with fewer frames (the array keeps the first call's
contents).  One case is also checked against the FP64 oracle at the sensor's
slope bound.  A slice that does not fit the array is rejected on the host."""
import numpy as np
import pytest

from synth.configs import CFG1, CFG2, ATMO1, ATMO2, SensorConfig
from synth.screens import open_loop_batch
import oracle
from tests.gpu_common import torch_cuda, say, check_frame

pytestmark = pytest.mark.gpu

CFG_DET7 = SensorConfig(name="p32_det7_k12_obs_norm1", n_fft=128, n_pupil=32, n_bin=1, n_mod=12,
                        mod_radius_lod=2.5, wavelength_m=750e-9, diameter_m=8.0, obstruction=0.2,
                        norm_mode=1, det_window=7)
CFG_STOP8 = SensorConfig(name="p32_k12_stop8_obs_norm1", n_fft=128, n_pupil=32, n_bin=2, n_mod=12,
                         mod_radius_lod=2.5, wavelength_m=750e-9, diameter_m=8.0, obstruction=0.2,
                         norm_mode=1, field_stop_lod=8.0)


def _pair(plan, opd, want_pupils, frame0=None):
    """(pupils, slopes) of pwfs_measure and of pwfs_measure_static."""
    torch = torch_cuda()
    B, S = opd.shape[0], plan.n_sub
    out = []
    for static in (False, True):
        pup = torch.full((B, 4, S, S), float("nan"), device="cuda") if want_pupils else None
        sl = torch.full((B, 2 * plan.n_valid), float("nan"), device="cuda")
        if frame0 is not None:
            plan.set_frame_counter(frame0)
        (plan.measure_static_into if static else plan.measure_into)(opd, pup, sl)
        torch.cuda.synchronize()
        out.append((None if pup is None else pup.cpu().numpy(), sl.cpu().numpy()))
    return out


@pytest.mark.parametrize("cfg,atmo,batch_max,sizes,want_pupils,detector", [
    (CFG1, ATMO1, 8, (7, 3), True, False),
    (CFG1, ATMO1, 4, (7, 2), False, True),
    (CFG2, ATMO2, 1, (2, 1), False, False),
    (CFG2, ATMO2, 2, (2, 1), True, False),
    (CFG_DET7, ATMO1, 3, (5, 2), True, False),
    (CFG_STOP8, ATMO1, 4, (5, 3), True, False),
], ids=["cfg1", "cfg1-detector-slices", "cfg2-b1", "cfg2-b2", "det-window", "field-stop"])
def test_static_equals_measure(cfg, atmo, batch_max, sizes, want_pupils, detector):
    import paper_1607_07624_amd as pw
    torch = torch_cuda()
    plan = pw.Plan(cfg, batch_max=batch_max)
    if detector:
        plan.set_detector(2.0e5, 1.0, seed=3)
    opd_all, _ = open_loop_batch(cfg, atmo, list(range(max(sizes))), r0_range=(0.08, 0.2),
                                 screen_n=64 if cfg.n_pupil == 32 else None)
    for call, B in enumerate(sizes):
        say(f"[gpu] static scratch {cfg.name} batch_max {batch_max}: call {call} with {B} frames")
        opd = torch.from_numpy(np.ascontiguousarray(opd_all[:B])).cuda()
        (p_ref, s_ref), (p_st, s_st) = _pair(plan, opd, want_pupils, frame0=1000 + call if detector else None)
        assert np.all(np.isfinite(s_st))
        assert np.array_equal(s_st, s_ref)
        if want_pupils:
            assert np.array_equal(p_st, p_ref)
    if cfg is CFG1 and not detector:
        # the static path against the oracle, at the sensor's bounds
        orc = oracle.Oracle(cfg)
        for i in range(sizes[-1]):
            p_o, s_o = orc.measure(opd_all[i].astype(np.float64))
            check_frame(f"{cfg.name} static frame {i}", s_st[i], s_o, p_st[i], p_o)
    plan.close()


def test_static_rejects_slices_beyond_the_array():
    import paper_1607_07624_amd as pw
    from paper_1607_07624_amd._lib import PwfsError
    torch = torch_cuda()
    plan = pw.Plan(CFG2, batch_max=4)      # 4 frames of 10.2 MB intermediate each: beyond 32 MiB
    opd = torch.zeros((4, CFG2.n_pupil, CFG2.n_pupil), device="cuda")
    sl = torch.zeros((4, 2 * plan.n_valid), device="cuda")
    with pytest.raises(PwfsError) as ei:
        plan.measure_static_into(opd, None, sl)
    assert ei.value.status == -2 and "bytes" in str(ei.value)
    # a slice of 2 frames fits: a 2-frame call goes through
    plan.measure_static_into(opd[:2], None, sl[:2])
    torch.cuda.synchronize()
    assert float(sl[:2].abs().max()) <= 1e-6
    plan.close()
