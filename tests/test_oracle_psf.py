"""Pins of the PSF reference (oracle/psf.py) against properties fixed by the
Fourier optics: the diffraction-limited peak, Parseval, the exact shift of a
whole-wave tilt, the point symmetry of a flat pupil's PSF, the conjugation
symmetry under phi -> -phi, and a brute-force DFT on a tiny grid."""
import numpy as np

import oracle
from oracle import psf as opsf


def _amp(P):
    return oracle.pupil_amplitude(P, 0.0)


def test_flat_peak_parseval_and_symmetry():
    A = _amp(32)
    p = opsf.psf(np.zeros((32, 32)), A, 1.65e-6, 4)
    N = 128
    assert abs(p[N // 2, N // 2] - 1.0) < 1e-13 and p.max() == p[N // 2, N // 2]
    # Parseval: sum |F|^2 = N^2 sum |E|^2
    assert abs(p.sum() - N * N * (A ** 2).sum() / A.sum() ** 2) < 1e-9 * p.sum()
    # a real, point-symmetric pupil has a point-symmetric PSF about (N/2, N/2)
    q = np.roll(np.flip(p, (0, 1)), (1, 1), (0, 1))
    assert np.allclose(p, q, atol=1e-13)


def test_whole_wave_tilt_shifts_by_pad_pixels():
    P, pad, lam = 32, 4, 1.0e-6
    A = _amp(P)
    x = np.arange(P)
    opd = np.tile(2.0 * x / P * lam * 1e9, (P, 1))            # two waves across the pupil in x
    p0 = opsf.psf(np.zeros((P, P)), A, lam, pad)
    p1 = opsf.psf(opd, A, lam, pad)
    assert np.allclose(p1, np.roll(p0, 2 * pad, axis=1), atol=1e-12)
    assert abs(opsf.strehl(opd, A, lam) - p1[pad * P // 2, pad * P // 2]) < 1e-12


def test_phase_conjugation_mirrors_the_psf():
    rng = np.random.default_rng(3)
    A = _amp(16)
    opd = rng.normal(0, 100.0, (16, 16))
    p = opsf.psf(opd, A, 1.0e-6, 2)
    m = opsf.psf(-opd, A, 1.0e-6, 2)
    assert np.allclose(m, np.roll(np.flip(p, (0, 1)), (1, 1), (0, 1)), atol=1e-12)


def test_brute_force_dft_tiny_grid():
    rng = np.random.default_rng(4)
    P, pad = 6, 2
    A = rng.uniform(0.5, 1.0, (P, P))
    opd = rng.normal(0, 200.0, (P, P))
    lam = 0.8e-6
    N = P * pad
    E = A * np.exp(2j * np.pi * opd * 1e-9 / lam)
    F = np.zeros((N, N), complex)
    for v in range(N):
        for u in range(N):
            F[v, u] = sum(E[y, x] * np.exp(-2j * np.pi * (v * y + u * x) / N) for y in range(P) for x in range(P))
    ref = np.abs(np.roll(F, (N // 2, N // 2), (0, 1))) ** 2 / A.sum() ** 2
    assert np.allclose(opsf.psf(opd, A, lam, pad), ref, rtol=1e-12, atol=1e-14)
