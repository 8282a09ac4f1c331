"""Pins of the detector reference (oracle/detector.py): the counter-based
generator against its published known-answer vectors, and the photon and
readout noise against the moments of the Poisson and normal laws."""
import os

import numpy as np
import pytest

from oracle import detector as det

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = det.philox4x32_10(*v[0:4], *v[4:6])
        assert [int(o) for o in out] == v[6:10]


def test_uniform_is_strictly_inside_the_unit_interval():
    u = det.uniform(np.array([0, 0xFFFFFFFF], np.uint64))
    assert u[0] == 2.0 ** -33 and u[1] == 1.0 - 2.0 ** -33


@pytest.mark.parametrize("lam,n", [(0.3, 20000), (4.0, 20000), (40.0, 20000), (700.0, 4000), (2500.0, 1500),
                                   (2.0e4, 20000)])
def test_poisson_moments(lam, n):
    """Sample mean within 4.5 standard errors of lam, sample variance within
    4.5 of its standard errors of lam (Poisson: var = mean; the fourth central
    moment gives Var(s^2) ~ (2 lam^2 + lam) / n).  700 and 2500 exercise the
    split into pieces of 500, 2e4 the normal approximation."""
    k = det.poisson_counts(np.full(n, lam), frame=11, seed=0x1234_5678_9ABC)
    m, v = k.mean(), k.var(ddof=1)
    assert abs(m - lam) <= 4.5 * np.sqrt(lam / n)
    assert abs(v - lam) <= 4.5 * np.sqrt((2 * lam * lam + lam) / n)
    if lam < 1.0:
        p0 = np.mean(k == 0)
        assert abs(p0 - np.exp(-lam)) <= 4.5 * np.sqrt(np.exp(-lam) * (1 - np.exp(-lam)) / n)


def test_poisson_zero_and_tiny_means():
    k = det.poisson_counts(np.array([0.0, 0.0, 1e-12, -1.0]), frame=0, seed=5)
    assert list(k) == [0, 0, 0, 0]


def test_gaussian_moments_and_frame_independence():
    n = 40000
    z = det.gaussians(n, frame=3, seed=99)
    assert abs(z.mean()) <= 4.5 / np.sqrt(n)
    assert abs(z.var() - 1.0) <= 4.5 * np.sqrt(2.0 / n)
    z2 = det.gaussians(n, frame=4, seed=99)
    assert abs(np.corrcoef(z, z2)[0, 1]) <= 4.5 / np.sqrt(n)
    assert np.array_equal(z, det.gaussians(n, frame=3, seed=99))
    assert not np.array_equal(z, det.gaussians(n, frame=3, seed=100))


def test_detect_photon_budget_and_integers():
    rng = np.random.default_rng(1)
    I = rng.uniform(0.0, 2.0, size=(3, 4, 8, 8)).astype(np.float32)
    px = det.detect(I, gain=50.0, ron_e=0.0, seed=7, frame0=100)
    assert np.array_equal(px, np.round(px))                    # no readout noise: whole electrons
    tot = 50.0 * I.astype(np.float64).sum()
    assert abs(px.astype(np.float64).sum() - tot) <= 4.5 * np.sqrt(tot)
    again = det.detect(I, gain=50.0, ron_e=0.0, seed=7, frame0=100)
    assert np.array_equal(px, again)
    shifted = det.detect(I[1:], gain=50.0, ron_e=0.0, seed=7, frame0=101)
    assert np.array_equal(px[1:], shifted)                     # frame b uses index frame0 + b
    noisy = det.detect(I, gain=50.0, ron_e=1.0, seed=7, frame0=100)
    d = (noisy - px).astype(np.float64).ravel()
    assert abs(d.mean()) <= 4.5 / np.sqrt(d.size) and abs(d.std() - 1.0) <= 0.1
