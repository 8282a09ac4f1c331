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
