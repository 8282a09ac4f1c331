"""Pins of the FP64 oracle against things it does not compute itself.

Brute-force DFT matrices, exact symmetries of the optics, identity and
single-face special cases with closed-form answers, flux conservation
through a unit-modulus mask, the geometric-optics limit of the modulated
pyramid's tilt response, and the separable (row/column) factorisation of
the 2-D operator.  All run on the CPU.
"""
import numpy as np
import pytest

from synth.configs import SensorConfig, CFG1, CFG2
from synth.screens import tilt_opd_nm, open_loop_batch
from synth.configs import ATMO1
import oracle
from oracle import pwfs as opw

TINY = SensorConfig(name="tiny", n_fft=16, n_pupil=4, n_bin=2, n_mod=8,
                    mod_radius_lod=1.0, wavelength_m=750e-9, diameter_m=1.0)
TINY24 = SensorConfig(name="tiny24", n_fft=24, n_pupil=6, n_bin=3, n_mod=12,
                      mod_radius_lod=1.5, wavelength_m=750e-9, diameter_m=1.0)
SMALL = SensorConfig(name="small", n_fft=64, n_pupil=16, n_bin=2, n_mod=8,
                     mod_radius_lod=3.0, wavelength_m=750e-9, diameter_m=2.0)


def _signed(n, N):
    return n if n < N // 2 else n - N


def brute_intensity(cfg, opd_nm, A):
    """Explicit DFT matrices, mask as exact powers of -i (Delta = N/4)."""
    N, P, K = cfg.n_fft, cfg.n_pupil, cfg.n_mod
    assert cfg.delta * 4 == N
    o = (N - P) // 2
    idx = np.arange(N)
    W = np.exp(-2j * np.pi * np.outer(idx, idx) / N)
    Wi = np.conj(W)
    powers = np.array([1, -1j, -1, 1j])
    M = np.empty((N, N), complex)
    for v in range(N):
        for u in range(N):
            M[v, u] = powers[(abs(_signed(u, N)) + abs(_signed(v, N))) % 4]
    rho = cfg.mod_radius_lod * N / P
    xc = (N - 1) / 2
    I = np.zeros((N, N))
    for k in range(K):
        th = 2 * np.pi * k / K
        a, b = rho * np.cos(th), rho * np.sin(th)
        E = np.zeros((N, N), complex)
        for y in range(P):
            for x in range(P):
                Y, X = o + y, o + x
                ph = 2 * np.pi * opd_nm[y, x] * 1e-9 / cfg.wavelength_m
                ph += 2 * np.pi * (a * (X - xc) + b * (Y - xc)) / N
                E[Y, X] = A[y, x] * np.exp(1j * ph)
        F = W @ E @ W
        Eo = Wi @ (M * F) @ Wi / N ** 2
        I += np.abs(Eo) ** 2
    return I / K


@pytest.mark.parametrize("N", [8, 12, 16, 20, 32])
def test_fft2_matches_dft_matrix(N):
    import scipy.fft as sfft
    rng = np.random.default_rng(N)
    x = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    idx = np.arange(N)
    W = np.exp(-2j * np.pi * np.outer(idx, idx) / N)
    assert np.abs(sfft.fft2(x) - W @ x @ W).max() < 1e-12 * N * N
    assert np.abs(sfft.ifft2(x) - np.conj(W) @ x @ np.conj(W) / N ** 2).max() < 1e-13 * N


@pytest.mark.parametrize("cfg", [TINY, TINY24])
def test_intensity_matches_brute_force(cfg):
    rng = np.random.default_rng(7)
    A = opw.pupil_amplitude(cfg.n_pupil)
    opd = rng.normal(0, 300.0, (cfg.n_pupil, cfg.n_pupil))
    ref = brute_intensity(cfg, opd, A)
    got = opw.intensity(cfg, opd, A)
    assert np.abs(got - ref).max() <= 1e-12 * ref.max()


def test_pupil_amplitude_small_cases():
    # P = 4: radius 2 about (1.5, 1.5); only the four corners (r^2 = 4.5) are out.
    A4 = opw.pupil_amplitude(4)
    exp4 = np.ones((4, 4)); exp4[0, 0] = exp4[0, 3] = exp4[3, 0] = exp4[3, 3] = 0
    assert np.array_equal(A4, exp4)
    assert opw.pupil_amplitude(2).sum() == 4
    for P in (32, 160):
        A = opw.pupil_amplitude(P)
        assert np.array_equal(A, A[::-1]) and np.array_equal(A, A[:, ::-1]) and np.array_equal(A, A.T)
        # Area of a disc of radius P/2 up to a perimeter-sized error.
        assert abs(A.sum() - np.pi * P * P / 4) < np.pi * P
    Ao = opw.pupil_amplitude(160, 0.2)
    c = 79.5
    assert Ao[80, 80] == 0 and Ao[80, 80 + 16] == 1  # r = 0.5 (inside stop), r = 16.5 (> 16)


def test_valid_subapertures_small_case():
    A = np.zeros((4, 4))
    A[0:2, 0:2] = [[1, 1], [0, 0]]      # fill 0.5 -> valid (tie counts)
    A[0:2, 2:4] = [[1, 0], [0, 0]]      # fill 0.25 -> invalid
    A[2:4, 0:2] = 1                     # full
    assert list(opw.valid_subapertures(A, 2)) == [0, 2]
    # Circle of P = 4 binned 2 x 2: each quadrant has 3 of 4 pixels lit.
    assert list(opw.valid_subapertures(opw.pupil_amplitude(4), 2)) == [0, 1, 2, 3]


def test_slopes_hand_values():
    p = np.zeros((4, 2, 2))
    p[0], p[1], p[2], p[3] = 1.0, 3.0, 1.0, 3.0
    p[:, 1, 1] = [2.0, 2.0, 0.0, 4.0]   # subap 3: total 8, sx = 4/8, sy = 0
    s = opw.slopes(p, np.array([0, 3]))
    assert np.allclose(s, [0.5, 0.5, 0.0, 0.0])
    s1 = opw.slopes(p * 10, np.array([0, 3]), norm_mode=1)
    assert np.allclose(s1, [0.5, 0.5, 0.0, 0.0])
    # Global normalisation uses the mean total flux over V only.
    p2 = p.copy(); p2[:, 0, 1] = 100.0
    assert np.allclose(opw.slopes(p2, np.array([0, 3])), s)


@pytest.mark.parametrize("cfg", [TINY, SMALL, CFG1])
def test_flux_conserved_through_mask(cfg):
    rng = np.random.default_rng(3)
    A = opw.pupil_amplitude(cfg.n_pupil)
    opd = rng.normal(0, 500.0, (cfg.n_pupil, cfg.n_pupil))
    I = opw.intensity(cfg, opd, A)
    assert abs(I.sum() - (A ** 2).sum()) <= 1e-12 * A.sum()
    # The four windows hold most of it, never more than all of it.
    pup = opw.pupil_images(cfg, I)
    assert pup.sum() <= I.sum() * (1 + 1e-12) and pup.sum() > 0.5 * I.sum()


def test_identity_mask_returns_pupil_intensity():
    cfg = SMALL
    rng = np.random.default_rng(4)
    A = opw.pupil_amplitude(cfg.n_pupil)
    opd = rng.normal(0, 400.0, (cfg.n_pupil, cfg.n_pupil))
    N, P = cfg.n_fft, cfg.n_pupil
    o = (N - P) // 2
    I = opw.intensity(cfg, opd, A, mask=np.ones((N, N)))
    ref = np.zeros((N, N)); ref[o:o + P, o:o + P] = A ** 2
    assert np.abs(I - ref).max() < 1e-13


def test_single_face_is_pure_shift():
    cfg = SMALL
    N, P, d = cfg.n_fft, cfg.n_pupil, cfg.delta
    o = (N - P) // 2
    rng = np.random.default_rng(5)
    A = opw.pupil_amplitude(P)
    opd = rng.normal(0, 400.0, (P, P))
    u = np.arange(N)
    face = np.exp(-2j * np.pi * d * (u[None, :] + u[:, None]) / N)
    I = opw.intensity(cfg, opd, A, mask=face)
    ref = np.zeros((N, N)); ref[o + d:o + d + P, o + d:o + d + P] = A ** 2
    assert np.abs(I - ref).max() < 1e-13
    pup = opw.pupil_images(cfg, I)
    b = cfg.n_bin
    S = P // b
    assert np.abs(pup[3] - A.reshape(S, b, S, b).sum(axis=(1, 3))).max() < 1e-12
    assert np.abs(pup[:3]).max() < 1e-12


@pytest.mark.parametrize("cfg", [SMALL, CFG1])
def test_flat_wavefront_symmetries(cfg):
    orc = oracle.Oracle(cfg)
    p = orc.ref_pupils
    scale = p.max()
    # x-mirror maps the -x pupils onto the +x pupils, y-mirror likewise,
    # and with K % 4 == 0 the modulation ring is symmetric under x <-> y.
    assert np.abs(p[1] - p[0][:, ::-1]).max() <= 1e-13 * scale
    assert np.abs(p[2] - p[0][::-1, :]).max() <= 1e-13 * scale
    assert np.abs(p[3] - p[0][::-1, ::-1]).max() <= 1e-13 * scale
    assert np.abs(p[0] - p[0].T).max() <= 1e-13 * scale
    fl = p.reshape(4, -1).sum(1)
    assert np.ptp(fl) <= 1e-13 * fl.mean()
    nv = orc.n_valid
    sx, sy = orc.s_ref[:nv], orc.s_ref[nv:]
    assert abs(sx.sum()) < 1e-12 and abs(sy.sum()) < 1e-12
    S = cfg.n_sub
    gx = np.zeros(S * S); gy = np.zeros(S * S)
    gx[orc.valid] = sx; gy[orc.valid] = sy
    gx = gx.reshape(S, S); gy = gy.reshape(S, S)
    assert np.abs(gx + gx[:, ::-1]).max() < 1e-12      # antisymmetric under the x-mirror
    assert np.abs(gx - gy.T).max() < 1e-12              # sx(ix, iy) = sy(iy, ix)


def _mean_sx(orc, alpha, axis="x"):
    cfg = orc.cfg
    opd = tilt_opd_nm(cfg.n_pupil, alpha, cfg.wavelength_m, axis)
    _, s = orc.measure(opd)
    nv = orc.n_valid
    return s[:nv], s[nv:]


def test_tilt_response_odd_linear_and_geometric():
    cfg = SMALL
    orc = oracle.Oracle(cfg)
    S = cfg.n_sub
    mirror = np.zeros(S * S, np.int64)
    for iy in range(S):
        for ix in range(S):
            mirror[iy * S + ix] = iy * S + (S - 1 - ix)
    pos = {j: i for i, j in enumerate(orc.valid)}
    mi = np.array([pos[mirror[j]] for j in orc.valid])
    sxp, syp = _mean_sx(orc, 0.3)
    sxm, _ = _mean_sx(orc, -0.3)
    assert np.abs(sxm + sxp[mi]).max() < 1e-12
    assert sxp.mean() > 0                         # +d phi / dx -> +sx
    assert abs(syp.mean()) < 1e-12                 # no cross-talk on average
    a = 0.01
    r1 = _mean_sx(orc, a)[0].mean()
    r2 = _mean_sx(orc, 2 * a)[0].mean()
    assert abs(r2 / r1 - 2.0) < 1e-3
    # y tilt gives the transposed response.
    _, syy = _mean_sx(orc, 0.3, axis="y")
    assert abs(syy.mean() - sxp.mean()) < 1e-12


def _row_op(N, d):
    """1-D operator T = IFFT diag(m) FFT with m(u) = exp(-2 pi i d |u_s| / N)."""
    us = np.abs(np.fft.fftfreq(N, 1.0 / N))
    m = np.exp(-2j * np.pi * d * us / N)
    return lambda f, ax: np.fft.ifft(np.fft.fft(f, axis=ax) * np.expand_dims(m, 1 - ax), axis=ax)


@pytest.mark.parametrize("cfg", [TINY24, SMALL])
def test_separable_factorisation_equals_literal(cfg):
    """Mask and tilt are separable, so the 2-D route equals the row then
    column 1-D route; this is the reordering the fast path relies on."""
    N, P = cfg.n_fft, cfg.n_pupil
    o = (N - P) // 2
    rng = np.random.default_rng(9)
    A = opw.pupil_amplitude(P)
    opd = rng.normal(0, 600.0, (P, P))
    E = np.zeros((N, N), complex)
    E[o:o + P, o:o + P] = A * np.exp(2j * np.pi * opd * 1e-9 / cfg.wavelength_m)
    T = _row_op(N, cfg.delta)
    rho = cfg.mod_radius_lod * N / P
    g = np.arange(N) - (N - 1) / 2
    I = np.zeros((N, N))
    for k in range(cfg.n_mod):
        th = 2 * np.pi * k / cfg.n_mod
        ra = np.exp(2j * np.pi * rho * np.cos(th) * g / N)
        rb = np.exp(2j * np.pi * rho * np.sin(th) * g / N)
        rows = T(E * ra[None, :], 1)
        out = T(rows * rb[:, None], 0)
        I += np.abs(out) ** 2
    I /= cfg.n_mod
    ref = opw.intensity(cfg, opd, A)
    assert np.abs(I - ref).max() < 1e-13 * max(1.0, ref.max())


GEO = SensorConfig(name="geo", n_fft=128, n_pupil=32, n_bin=2, n_mod=32,
                   mod_radius_lod=6.0, wavelength_m=750e-9, diameter_m=1.0)


def test_tilt_gain_geometric_optics_limit():
    """With a ring of many points and a radius of several lambda/D, a spot
    offset alpha spends a fraction 1/2 + arcsin(alpha / r) / pi of the
    cycle on the + faces, so the mean sx tends to (2/pi) arcsin(alpha / r);
    beyond the radius the spot never crosses the edge and sx saturates.
    A wrong tilt scale (rho) or face assignment fails this."""
    orc = oracle.Oracle(GEO)
    r = GEO.mod_radius_lod
    for alpha in (1.0, 2.0, 3.0, 4.5):
        got = _mean_sx(orc, alpha)[0].mean()
        geo = 2 / np.pi * np.arcsin(alpha / r)
        assert 0.9 * geo < got < 1.1 * geo, (alpha, got, geo)
    assert _mean_sx(orc, 1.5 * r)[0].mean() > 0.9


def test_cfg_counts():
    # Valid subapertures and pupil pixels of the two measured geometries.
    for cfg, npix, nv in ((CFG1, 812, 208), (CFG2, 20108, 1272)):
        A = opw.pupil_amplitude(cfg.n_pupil)
        assert A.sum() == npix
        assert opw.valid_subapertures(A, cfg.n_bin).size == nv


def test_random_screen_slopes_reference_subtracted():
    orc = oracle.Oracle(CFG1)
    opd, _ = open_loop_batch(CFG1, ATMO1, [0], screen_n=64)
    p, s = orc.measure(opd[0])
    _, s0 = orc.measure(np.zeros_like(opd[0]))
    assert np.abs(s0).max() < 1e-15
    assert np.isfinite(s).all() and np.abs(s).max() > 1e-3


@pytest.mark.parametrize("cfg", [TINY24, SMALL, CFG1])
def test_response_is_odd_in_phase(cfg):
    """With Delta = N/4 the conjugate mask equals the mask times (-1)^u, a
    shift by N/2 = 2 Delta, so conj(T g) is T conj(g) moved from one window
    to the other.  For a real pupil and a modulation ring symmetric in the
    x tilt this makes every subaperture's slopes exactly odd in the phase,
    s(-phi) = -s(phi), and the flat-wavefront reference exactly zero."""
    orc = oracle.Oracle(cfg)
    rng = np.random.default_rng(11)
    opd = rng.normal(0, 300.0, (cfg.n_pupil, cfg.n_pupil))
    _, sp = orc.measure(opd)
    _, sm = orc.measure(-opd)
    assert np.abs(sp + sm).max() <= 1e-12 * np.abs(sp).max()
    assert np.abs(orc.s_ref).max() < 1e-13
    pp = orc.pupils(opd)
    pm = orc.pupils(-opd)
    # Pupil-level statement: I_q(phi) = I_(q xor 1 xor 2)(-phi)
    for q in range(4):
        assert np.abs(pp[q] - pm[q ^ 3]).max() <= 1e-12 * pp.max()
