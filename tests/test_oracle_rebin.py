"""Pins of the oracle's detector resampling (the paper's pyramid output
resolution with pupils pup_diam pixels across, pup_dist apart: a
non-integer rebin) and of its pupil acquisition (Sec. 4 calibration)."""
import numpy as np
import pytest

import oracle
from synth.configs import SensorConfig, paper_pupil


def test_integer_pitch_is_the_block_sum():
    rng = np.random.default_rng(3)
    win = rng.random((32, 32))
    for b in (1, 2, 4, 8):
        S = 32 // b
        np.testing.assert_allclose(oracle.rebin(win, S), win.reshape(S, b, S, b).sum(axis=(1, 3)),
                                   rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("P,S", [(20, 9), (32, 7), (160, 36), (32, 31)])
def test_rebin_equals_supersampled_block_sums(P, S):
    """Split every pupil pixel into S x S equal parts: detector pixel (j, i)
    then covers exactly the P x P block of parts starting at (j P, i P)."""
    rng = np.random.default_rng(P * 100 + S)
    win = rng.random((P, P))
    fine = np.kron(win, np.ones((S, S))) / (S * S)
    brute = fine.reshape(S, P, S, P).sum(axis=(1, 3))
    np.testing.assert_allclose(oracle.rebin(win, S), brute, rtol=1e-12, atol=1e-12)


def test_rebin_conserves_flux_and_maps_constants():
    rng = np.random.default_rng(5)
    win = rng.random((160, 160))
    out = oracle.rebin(win, 36)
    assert abs(out.sum() - win.sum()) <= 1e-9 * win.sum()
    c = oracle.rebin(np.full((160, 160), 2.5), 36)
    np.testing.assert_allclose(c, 2.5 * (160 / 36) ** 2, rtol=1e-13)
    W = oracle.overlap_matrix(160, 36)
    np.testing.assert_allclose(W.sum(axis=1), 160 / 36, rtol=1e-13)   # every pixel is P/S wide
    np.testing.assert_allclose(W.sum(axis=0), 1.0, rtol=1e-13)        # every pupil pixel lands once


def test_valid_rule_at_integer_pitch_matches_block_rule():
    A = oracle.pupil_amplitude(64, 0.2)
    for b in (2, 4, 8):
        assert np.array_equal(oracle.valid_subapertures(A, 1, 64 // b), oracle.valid_subapertures(A, b))


def test_paper_geometry_valid_count_and_symmetry():
    """pup_diam 30 / pup_dist 36 on P = 160: the pupil image is a disc of 30
    detector pixels across inside each 36-pixel window; the fill rule keeps
    the pixels whose footprint is at least half inside it (about pi 15^2)."""
    A = paper_pupil(160, 30, 36).astype(np.float64)
    v = oracle.valid_subapertures(A, 1, 36)
    m = np.zeros(36 * 36, bool)
    m[v] = True
    m = m.reshape(36, 36)
    assert abs(v.size - np.pi * 15 ** 2) < 0.03 * np.pi * 15 ** 2
    assert np.array_equal(m, m[::-1]) and np.array_equal(m, m[:, ::-1]) and np.array_equal(m, m.T)
    assert not m[:3].any() and not m[-3:].any()       # 3-pixel dark border in the 36-pixel window


def test_acquisition_on_a_flat_frame_finds_the_pupil():
    """The paper's acquisition: flat wavefront, modulation radius raised to
    20 lambda/D, threshold.  On a small geometry the acquired set holds every
    fully illuminated detector pixel and differs from the geometric fill rule
    only on the rim."""
    cfg = SensorConfig(name="p32_acq", n_fft=128, n_pupil=32, n_bin=1, n_mod=128, mod_radius_lod=20.0,
                       wavelength_m=750e-9, diameter_m=8.0, det_window=9)
    A = paper_pupil(32, 30, 36).astype(np.float64)
    pup = oracle.pupil_images(cfg, oracle.intensity(cfg, np.zeros((32, 32)), A))
    acq = oracle.acquire_valid(pup, 0.5)
    geo = oracle.valid_subapertures(A, 1, 9)
    full = np.flatnonzero((oracle.rebin(A, 9) / (32 / 9) ** 2).ravel() >= 1.0 - 1e-12)
    assert set(full) <= set(acq)
    assert len(set(acq) ^ set(geo)) <= 8
