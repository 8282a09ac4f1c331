"""Pins of the oracle's circular field stop (Tab. 1 "pyramid": fov)."""
import numpy as np

import oracle
from synth.configs import SensorConfig

CFG = SensorConfig(name="p8_n32_k4", n_fft=32, n_pupil=8, n_bin=1, n_mod=4, mod_radius_lod=1.5,
                   wavelength_m=750e-9, diameter_m=8.0)


def _opd(P, seed):
    return np.random.default_rng(seed).standard_normal((P, P)) * 120.0


def test_stop_larger_than_the_grid_changes_nothing():
    opd = _opd(8, 1)
    a = oracle.intensity(CFG, opd)
    b = oracle.intensity(CFG.with_(field_stop_lod=1e3), opd)
    assert np.array_equal(a, b)


def test_stop_against_a_brute_force_dft():
    """Literal 2-D DFT sums (matrix form, not an FFT) with the stop applied."""
    cfg = CFG.with_(field_stop_lod=3.0)
    N, P = cfg.n_fft, cfg.n_pupil
    A = oracle.pupil_amplitude(P)
    opd = _opd(P, 2)
    o = (N - P) // 2
    E = np.zeros((N, N), complex)
    E[o:o + P, o:o + P] = A * np.exp(2j * np.pi * opd * 1e-9 / cfg.wavelength_m)
    n = np.arange(N)
    Fm = np.exp(-2j * np.pi * np.outer(n, n) / N)
    us = np.where(n < N // 2, n, n - N)
    R = 0.5 * 3.0 * N / P
    M = np.exp(-2j * np.pi * cfg.delta * (np.abs(us)[None, :] + np.abs(us)[:, None]) / N)
    M = M * ((us[None, :] ** 2 + us[:, None] ** 2) <= R * R)
    a, b = oracle.modulation_offsets(cfg)
    g = n - (N - 1) / 2.0
    I = np.zeros((N, N))
    for ak, bk in zip(a, b):
        ramp = np.exp(2j * np.pi * (ak * g[None, :] + bk * g[:, None]) / N)
        F = Fm @ (E * ramp) @ Fm
        back = np.conj(Fm) @ (M * F) @ np.conj(Fm) / N ** 2
        I += np.abs(back) ** 2
    np.testing.assert_allclose(oracle.intensity(cfg, opd), I / len(a), rtol=1e-10, atol=1e-14)


def test_energy_falls_as_the_stop_closes_and_flat_pupils_stay_symmetric():
    opd = _opd(8, 3)
    tot = [oracle.intensity(CFG.with_(field_stop_lod=d), opd).sum() for d in (1e3, 12.0, 6.0, 3.0, 1.0)]
    A = oracle.pupil_amplitude(8)
    assert tot[0] <= (A ** 2).sum() * (1 + 1e-12)
    assert all(x >= y for x, y in zip(tot, tot[1:])) and tot[-1] < 0.9 * tot[0]
    cfg = CFG.with_(field_stop_lod=4.0, n_mod=8)
    p = oracle.pupil_images(cfg, oracle.intensity(cfg, np.zeros((8, 8))))
    np.testing.assert_allclose(p[1], p[0][:, ::-1], rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(p[2], p[0][::-1, :], rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(p[3], p[0][::-1, ::-1], rtol=1e-9, atol=1e-15)


def test_stop_disc_membership_hand_counted():
    """The stop's diameter d (lambda/D) is a disc of radius R = d N / (2 P)
    focal pixels (one lambda/D is N / P pixels of the N-point grid).
    Counted by hand on the integer lattice, N = 32, P = 8 (4 pixels per
    lambda/D): d = 0.75 -> R = 1.5, u^2 + v^2 <= 2.25 keeps the centre, its 4
    edge and 4 corner neighbours (9 bins); d = 1 -> R = 2 adds (+-2, 0) and
    (0, +-2) (13 bins); d = 2 -> R = 4: 49 bins (1 + 4 x 12 lattice points with
    0 < u^2 + v^2 <= 16 in the four quadrants).  Reading d as a radius
    (R = d N / P) would give 29, 49 and 197."""
    N, P = 32, 8
    for d, count in ((0.75, 9), (1.0, 13), (2.0, 49)):
        m = oracle.field_stop_mask(N, P, d)
        assert int(m.sum()) == count, (d, int(m.sum()))
        assert m[0, 0] == 1.0                                        # apex bin (frequency 0) is inside
    m = oracle.field_stop_mask(N, P, 0.75)
    assert m[1, 1] == 1.0 and m[N - 1, N - 1] == 1.0 and m[0, 2] == 0.0 and m[2, 0] == 0.0


def test_stop_transmits_the_airy_encircled_energy():
    """Physical pin of the stop's size: a flat circular pupil (P = 64, N = 4P),
    no pyramid, no modulation, mask = stop alone.  The flux back in the pupil
    plane is the PSF energy inside the stop, which for a filled circular
    aperture is the Airy encircled energy 1 - J0(pi rho)^2 - J1(pi rho)^2 at
    radius rho = d / 2 lambda/D (Born and Wolf, Sec. 8.5.2).  Discretisation:
    the focal plane is sampled at 4 points per lambda/D and the pupil is a
    64-pixel digital circle; near the stop's edge the encircled energy grows
    by about 0.04 per focal pixel of radius at rho = 1 and less beyond, so a
    lattice disc whose effective radius is within a fraction of a pixel of R
    stays within 5e-3 of the continuous value.  Reading the diameter as a
    radius changes the value by 0.024 to 0.08 at these sizes."""
    from scipy.special import j0, j1
    P = 64
    cfg = SensorConfig(name="airy_p64", n_fft=4 * P, n_pupil=P, n_bin=1, n_mod=1, mod_radius_lod=0.0,
                       wavelength_m=750e-9, diameter_m=8.0)
    A = oracle.pupil_amplitude(P)
    for d in (2.0, 3.0, 4.0, 6.0, 8.0):
        stop = oracle.field_stop_mask(cfg.n_fft, P, d).astype(complex)
        ee = oracle.intensity(cfg, np.zeros((P, P)), A, mask=stop).sum() / A.sum()
        rho = 0.5 * d
        airy = 1.0 - j0(np.pi * rho) ** 2 - j1(np.pi * rho) ** 2
        assert abs(ee - airy) <= 5e-3, (d, ee, airy)


def test_stop_blocks_a_psf_tilted_outside_it():
    """A flat wavefront tilted by t lambda/D puts the PSF core t lambda/D off
    axis (t N / P focal pixels).  A stop of diameter 2t + 1 lambda/D (edge
    half a lambda/D beyond the core) passes most of the light; one of 2t - 1
    (edge half a lambda/D short of it) passes only the Airy wings."""
    from synth.screens import tilt_opd_nm
    P = 64
    cfg = SensorConfig(name="tilt_p64", n_fft=4 * P, n_pupil=P, n_bin=1, n_mod=1, mod_radius_lod=0.0,
                       wavelength_m=750e-9, diameter_m=8.0)
    A = oracle.pupil_amplitude(P)
    for t in (3.0, 5.0):
        opd = tilt_opd_nm(P, t, cfg.wavelength_m, "x")
        ee = {}
        for d in (2 * t + 1, 2 * t - 1):
            stop = oracle.field_stop_mask(cfg.n_fft, P, d).astype(complex)
            ee[d] = oracle.intensity(cfg, opd, A, mask=stop).sum() / A.sum()
        assert ee[2 * t + 1] > 0.7 and ee[2 * t - 1] < 0.15, (t, ee)
