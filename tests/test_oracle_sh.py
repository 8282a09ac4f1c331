"""Pins of the Shack-Hartmann reference (oracle/sh.py): brute-force DFT of a
subaperture, zero slopes for a flat wavefront, the exact centroid of a
phase with one whole wave of tilt per padded box (a circular shift by pad
pixels per wave), the small-tilt gain pad * (waves across the subaperture),
and the mirror symmetry."""
import numpy as np

from oracle.sh import ShackHartmann


def test_spot_brute_force_dft():
    rng = np.random.default_rng(0)
    sh = ShackHartmann(8, 2, 2, 1e-6)
    opd = rng.normal(0, 150.0, (8, 8))
    sp = sh.spots(opd)
    s, M = sh.s, sh.M
    E = sh.A * np.exp(2j * np.pi * opd * 1e-9 / sh.lam)
    j = sh.valid[0]
    iy, ix = divmod(int(j), sh.n_sub)
    e = E[iy * s:(iy + 1) * s, ix * s:(ix + 1) * s]
    for v in range(M):
        for u in range(M):
            f = sum(e[y, x] * np.exp(-2j * np.pi * ((v - M // 2) * y + (u - M // 2) * x) / M)
                    for y in range(s) for x in range(s))
            assert abs(sp[0, v, u] - abs(f) ** 2) < 1e-10


def test_flat_is_zero_and_tilt_gain():
    sh = ShackHartmann(32, 8, 4, 1e-6)
    assert np.abs(sh.measure(np.zeros((32, 32)))[1]).max() < 1e-12
    # small tilt: alpha waves across each subaperture (s pixels) -> centroid shift ~ pad * alpha pixels
    alpha = 0.05
    x = np.arange(32)
    opd = np.tile(alpha * x / sh.s * sh.lam * 1e9, (32, 1))
    s = sh.measure(opd)[1]
    n = sh.n_valid
    full = [i for i, j in enumerate(sh.valid) if sh.A.reshape(8, 4, 8, 4)[j // 8, :, j % 8, :].min() > 0]
    g = s[:n][full] / (sh.pad * alpha)
    assert np.all(np.abs(g - 1.0) < 0.05)
    assert np.abs(s[n:][full]).max() < 1e-9


def test_mirror_symmetry():
    """Mirroring the wavefront in x inside every subaperture mirrors each spot
    about the zero frequency: spot'[v, u] = spot[v, (M - u) mod M] exactly
    on fully illuminated subapertures, and its centroid changes sign up
    to the unpaired column u = 0: cx + cx' = -M * (fraction of light in u = 0)."""
    rng = np.random.default_rng(1)
    sh = ShackHartmann(32, 8, 2, 1e-6)
    opd = rng.normal(0, 80.0, (32, 32))
    s = sh.s
    mirrored = opd.reshape(32, 8, s)[:, :, ::-1].reshape(32, 32)      # mirror inside each subaperture
    full = np.array([sh.A.reshape(8, s, 8, s)[j // 8, :, j % 8, :].min() > 0 for j in sh.valid])
    a, b = sh.spots(opd)[full], sh.spots(mirrored)[full]        # amplitude symmetric inside these
    M = sh.M
    idx = (M - np.arange(M)) % M
    assert np.allclose(b, a[:, :, idx], rtol=1e-10, atol=1e-12 * a.max())
    c = np.arange(M) - M // 2
    cxa = (a * c).sum(axis=(1, 2)) / a.sum(axis=(1, 2))
    cxb = (b * c).sum(axis=(1, 2)) / b.sum(axis=(1, 2))
    frac0 = a[:, :, 0].sum(axis=1) / a.sum(axis=(1, 2))
    assert np.allclose(cxa + cxb, -M * frac0, atol=1e-10)
