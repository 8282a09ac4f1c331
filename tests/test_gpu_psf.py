"""PSF camera (zero-padded PSF of the residual wavefront, Strehl ratio,
long-exposure accumulation) through the C ABI against the FP64 reference in
oracle/psf.py.  Gate: PSF relative L2 error <= 1e-5 and max |error| <= 1e-6
of the diffraction-limited peak (FP32 transforms of length P and N = pad P);
Strehl ratios within 1e-6 absolute."""
import numpy as np
import pytest

from synth.configs import CFG1, CFG2, ATMO1, ATMO2
from synth.screens import open_loop_batch
import oracle
from oracle import psf as opsf
from tests.gpu_common import torch_cuda, rel_l2, say

pytestmark = pytest.mark.gpu


def _check(P, pad, lam, opd, batch_max):
    import paper_1607_07624_amd as pw
    torch = torch_cuda()
    cam = pw.PsfCamera(P, pad, lam, batch_max=batch_max)
    A = oracle.pupil_amplitude(P, 0.0)
    psf, sr = cam.compute(torch.from_numpy(np.ascontiguousarray(opd)).cuda())
    torch.cuda.synchronize()
    psf, sr = psf.cpu().numpy(), sr.cpu().numpy()
    for i in range(len(opd)):
        ref = opsf.psf(opd[i].astype(np.float64), A, lam, pad)
        e = rel_l2(psf[i], ref)
        m = float(np.abs(psf[i] - ref).max())
        s_ref = opsf.strehl(opd[i].astype(np.float64), A, lam)
        say(f"[gpu] psf P={P} pad={pad}: frame {i} rel err {e:.3e}, max abs {m:.3e}, "
            f"Strehl {sr[i]:.6f} (ref {s_ref:.6f})")
        assert e <= 1e-5 and m <= 1e-6
        assert abs(sr[i] - s_ref) <= 1e-6
        assert abs(psf[i][pad * P // 2, pad * P // 2] - s_ref) <= 1e-6
    return cam


def test_psf_small_grid_and_flat_peak():
    import paper_1607_07624_amd as pw
    torch = torch_cuda()
    opd, _ = open_loop_batch(CFG1, ATMO1, [60, 61, 62], screen_n=64)
    opd = np.concatenate([np.zeros((1, 32, 32), np.float32), 0.2 * opd])   # flat frame first
    cam = _check(32, 4, 1.65e-6, opd, batch_max=2)                          # slices of 2 (ragged tail)
    psf, sr = cam.compute(torch.zeros((1, 32, 32), device="cuda"))
    assert abs(float(psf[0, 64, 64]) - 1.0) <= 1e-6 and abs(float(sr[0]) - 1.0) <= 1e-6
    cam.close()
    _check(64, 2, 1.0e-6, 0.3 * open_loop_batch(
        type(CFG1)(name="p64", n_fft=256, n_pupil=64, n_bin=2, n_mod=4, mod_radius_lod=3.0,
                   wavelength_m=750e-9, diameter_m=8.0), ATMO1, [63], screen_n=64)[0], batch_max=1).close()


def test_psf_lbt_like_h_band():
    """160-pixel pupil, H band (1.65 um), padding 8: N = 1280."""
    opd, _ = open_loop_batch(CFG2, ATMO2, [70, 71])
    _check(160, 8, 1.65e-6, 0.05 * opd, batch_max=2).close()


def test_long_exposure_accumulation():
    import paper_1607_07624_amd as pw
    torch = torch_cuda()
    opd, _ = open_loop_batch(CFG1, ATMO1, [64, 65, 66, 67, 68], screen_n=64)
    opd = 0.2 * opd
    A = oracle.pupil_amplitude(32, 0.0)
    cam = pw.PsfCamera(32, 4, 1.65e-6, batch_max=2)
    d = torch.from_numpy(np.ascontiguousarray(opd)).cuda()
    start = torch.full((128, 128), 0.25, device="cuda")
    acc, _ = cam.compute(d, psf=start.clone(), accumulate=True)
    ref = 0.25 + sum(opsf.psf(o.astype(np.float64), A, 1.65e-6, 4) for o in opd)
    e = rel_l2(acc.cpu().numpy(), ref)
    say(f"[gpu] long exposure (5 frames, slices of 2): rel err {e:.3e}")
    assert e <= 1e-5
    cam.close()
