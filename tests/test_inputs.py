"""Checks of the seeded input generators (screens, frozen flow, KL modes)."""
import numpy as np

from synth.configs import CFG1, CFG2, ATMO1, ATMO2, AtmoConfig
from synth.screens import von_karman_opd_nm, frozen_flow_sequence, open_loop_batch
from synth.kl import kl_modes
from oracle.pwfs import pupil_amplitude


def test_structure_function_kolmogorov_small_separations():
    """Kolmogorov law D(r) = 6.88 (r / r0)^(5/3) rad^2 (r << L0).

    A band-limited FFT screen misses the power beyond Nyquist and below
    the grid frequency, so D sits 20-30 % under the law at a few pixels;
    a wrong variance normalisation (x2, x0.5) or wavelength scaling falls
    far outside the band checked here, and the 5/3 log-slope pins the
    spectral exponent."""
    n, dx, r0 = 512, 0.02, 0.1
    D = {2: [], 4: []}
    for seed in range(6):
        opd = von_karman_opd_nm(n, dx, r0, 1e4, np.random.default_rng(seed))
        ph = opd * 1e-9 * 2 * np.pi / 500e-9
        for s in D:
            D[s].append(np.mean((ph[:, s:] - ph[:, :-s]) ** 2))
    for s, v in D.items():
        theory = 6.88 * (s * dx / r0) ** (5.0 / 3.0)
        assert 0.65 < np.mean(v) / theory < 0.9, (s, np.mean(v), theory)
    slope = np.log2(np.mean(D[4]) / np.mean(D[2]))
    assert abs(slope - 5.0 / 3.0) < 0.15


def test_screens_seeded_and_float32():
    a, r0a = open_loop_batch(CFG1, ATMO1, [0, 1], screen_n=64)
    b, _ = open_loop_batch(CFG1, ATMO1, [0, 1], screen_n=64)
    assert a.dtype == np.float32 and a.shape == (2, 32, 32)
    assert np.array_equal(a, b) and not np.array_equal(a[0], a[1])
    c, r0c = open_loop_batch(CFG2, ATMO2, [3, 4], r0_range=(0.08, 0.2))
    assert c.shape == (2, 160, 160) and np.all((r0c >= 0.08) & (r0c <= 0.2))


def test_frozen_flow_translates_toward_plus_x():
    atmo = AtmoConfig(r0_m=0.12, L0_m=40.0, wind_m_s=CFG2.pixel_m * 1000.0 * 0.25)
    seq = frozen_flow_sequence(CFG2, atmo, 9, seed=2, screen_n=512)
    # 0.25 px per step: after 8 steps the pattern has moved by exactly 2 px.
    assert np.abs(seq[8][:, 2:] - seq[0][:, :-2]).max() < 1e-3 * np.abs(seq[0]).max()


def test_kl_modes_orthonormal_pistonfree_tiptilt_first():
    A = pupil_amplitude(32)
    B = kl_modes(A, CFG1.pixel_m, 25.0, 60, cache=False)
    n = int(A.sum())
    F = B.reshape(60, -1)
    assert np.abs(F @ F.T / n - np.eye(60)).max() < 1e-12
    assert np.abs(F.sum(axis=1)).max() < 1e-9
    assert np.abs(B[:, A == 0]).max() == 0.0
    x = (np.arange(32) - 15.5)[None, :] * np.ones((32, 1))
    tt = np.stack([x[A > 0], x.T[A > 0]])
    tt /= np.linalg.norm(tt, axis=1, keepdims=True)
    # The first two modes span tip and tilt almost entirely.
    for i in (0, 1):
        v = B[i][A > 0] / np.linalg.norm(B[i][A > 0])
        assert np.linalg.norm(tt @ v) > 0.98


def test_layered_opd_ground_layer_and_integer_shift():
    """Single ground layer: every direction sees the same crop.  A layer whose
    shift is a whole number of pixels is the shifted crop of the same screen
    (bilinear weights 0/1), with r0 scaled by fraction^(-3/5)."""
    from synth.configs import SensorConfig, AtmoConfig
    from synth.screens import layered_opd_nm, von_karman_opd_nm
    cfg = SensorConfig(name="t", n_fft=128, n_pupil=32, n_bin=2, n_mod=8, mod_radius_lod=3.0,
                       wavelength_m=750e-9, diameter_m=8.0)
    atmo = AtmoConfig(r0_m=0.2, L0_m=20.0)
    dirs = ((0.0, 0.0), (10.0, -5.0), (-7.0, 3.0))
    o = layered_opd_nm(cfg, atmo, ((0.0, 1.0),), dirs, seed=3, screen_n=128)
    assert np.array_equal(o[0], o[1]) and np.array_equal(o[0], o[2])
    arcsec = np.pi / (180 * 3600)
    h = 3 * cfg.pixel_m / (10.0 * arcsec)             # 10 arcsec -> exactly 3 px in x
    o2 = layered_opd_nm(cfg, atmo, ((h, 0.5),), ((10.0, 0.0),), seed=4, screen_n=128)
    scr = von_karman_opd_nm(128, cfg.pixel_m, 0.2 * 0.5 ** (-0.6), 20.0, np.random.default_rng(4), 500e-9)
    c = (128 - 32) // 2
    assert np.allclose(o2[0], scr[c:c + 32, c + 3:c + 35].astype(np.float32), atol=1e-3)
