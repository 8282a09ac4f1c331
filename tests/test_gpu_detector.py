"""Detector step (photon and readout noise on Philox4x32-10 counters) through
the C ABI against the FP64 reference in oracle/detector.py.

pwfs_detect on seeded synthetic images: the photon counts are integers
decided by IEEE products of the same uniforms on both sides, so they must
match exactly (ron = 0: bit-identical pixels); with readout noise the
Box-Muller deviates agree to a few float ulps.  In pwfs_measure the detector
must be reproducible per frame index, independent of batching, and equal to
pwfs_detect applied to the same noiseless images."""
import numpy as np
import pytest

from synth.configs import CFG1, CFG2, ATMO2, CFG4_R0_RANGE, photoelectrons_per_frame, DETECTOR_RON_E
from synth.screens import open_loop_batch
from oracle import detector as odet
from tests.gpu_common import torch_cuda, say

pytestmark = pytest.mark.gpu


def _images(S, B, seed):
    """Seeded synthetic intensity images spanning four decades, with a few
    pixels bright enough for the normal-approximation branch."""
    rng = np.random.default_rng(seed)
    I = (10.0 ** rng.uniform(-3.0, 1.5, size=(B, 4, S, S))).astype(np.float32)
    I[:, 0, 0, :3] = np.float32(500.0)
    I[:, 1, 2, 2] = np.float32(0.0)
    return I


@pytest.mark.parametrize("frame0", [1000, (1 << 32) + 5])
def test_detect_counts_match_reference_exactly(frame0):
    import paper_1607_07624_amd as pw
    torch = torch_cuda()
    plan = pw.Plan(CFG1, batch_max=4)
    plan.set_detector(electrons_per_frame=1.0)
    e_frame = 100.0 / plan.detector()["gain"]      # a gain of ~100 e- per unit intensity
    plan.set_detector(electrons_per_frame=e_frame, readout_noise_e=0.0, seed=0x5EED_1234_ABCD)
    g = plan.detector()["gain"]
    S = plan.n_sub
    I = _images(S, 3, seed=17)
    lam = g * I.astype(np.float64)
    say(f"[gpu] detector gain {g:.4f} e-/unit, lam range {lam.min():.2e} .. {lam.max():.2e}")
    assert lam.max() > 1e4 and np.sort(lam.ravel())[-10] < 1e4 and (lam > 500).sum() > 10
    px = plan.detect(torch.from_numpy(I).cuda(), frame0).cpu().numpy()
    ref = odet.detect(I, g, 0.0, 0x5EED_1234_ABCD, frame0)
    bad = int((px != ref).sum())
    say(f"[gpu] detect frame0={frame0}: {px.size} pixels, {bad} differ")
    assert bad == 0
    plan.set_detector(electrons_per_frame=e_frame, readout_noise_e=1.5, seed=0x5EED_1234_ABCD)
    px = plan.detect(torch.from_numpy(I).cuda(), frame0).cpu().numpy()
    ref = odet.detect(I, g, 1.5, 0x5EED_1234_ABCD, frame0)
    tol = 2.0 * np.spacing(np.abs(ref).astype(np.float32)) + 1e-6
    worst = float((np.abs(px - ref) / tol).max())
    say(f"[gpu] detect with readout noise: worst |diff| / (2 ulp) = {worst:.3f}")
    assert worst <= 1.0
    plan.close()


def test_measure_with_detector_cfg2():
    import paper_1607_07624_amd as pw
    torch = torch_cuda()
    B = 16
    e_frame = photoelectrons_per_frame(CFG2)
    opd, _ = open_loop_batch(CFG2, ATMO2, list(range(B)), r0_range=CFG4_R0_RANGE)
    d = torch.from_numpy(opd).cuda()
    plan = pw.Plan(CFG2, batch_max=B)
    a, k = plan.get_schedule(B)
    plan.set_schedule(B // 2, a, k)                 # same modulation chunks -> same noiseless images
    clean, s_clean = plan.measure(d)
    plan.set_detector(e_frame, DETECTOR_RON_E, seed=2024)
    g = plan.detector()["gain"]
    px, s = plan.measure(d)
    assert plan.detector()["next_frame"] == B
    plan.set_frame_counter(0)
    px2, s2 = plan.measure(d)
    assert torch.equal(px, px2) and torch.equal(s, s2)
    plan.set_frame_counter(0)
    pa, sa = plan.measure(d[:B // 2].contiguous())
    pb, sb = plan.measure(d[B // 2:].contiguous())
    assert torch.equal(torch.cat([pa, pb]), px) and torch.equal(torch.cat([sa, sb]), s)
    direct = plan.detect(clean, 0)
    assert torch.equal(direct, px)
    # pixel noise: photon variance gain * I plus the readout variance
    c = clean.double().cpu().numpy() * g
    r = px.double().cpu().numpy() - c
    var_pred = float(c.mean() + DETECTOR_RON_E ** 2)
    say(f"[gpu] cfg2 detector: {e_frame:.3e} e-/frame, gain {g:.3f}, mean pixel {c.mean():.2f} e-, "
        f"noise mean {r.mean():.4f}, variance {r.var():.3f} (Poisson + readout {var_pred:.3f})")
    assert abs(r.mean()) <= 5 * np.sqrt(var_pred / r.size)
    assert abs(r.var() / var_pred - 1.0) <= 0.05
    dn = (s - s_clean).cpu().numpy()
    say(f"[gpu] slope noise RMS {dn.std():.4e} (signal RMS {s_clean.cpu().numpy().std():.4e})")
    assert 0.0 < dn.std() < s_clean.cpu().numpy().std()
    plan.close()
