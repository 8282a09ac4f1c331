"""Karhunen-Loeve modal basis of von Karman turbulence over the pupil.

This is the definition of the modal deformable mirror (its influence
functions), an input shared by both implementations; it holds none of the
sensor's arithmetic.

Modes are eigenvectors of the piston-removed phase covariance between
pupil pixels, C(r) proportional to (2 pi r / L0)^(5/6) K_(5/6)(2 pi r / L0)
(von Karman; the scale factor does not change eigenvectors).  The
covariance depends only on the pixel offset, so it is applied by FFT
convolution on a 2P x 2P grid; the leading eigenvectors are found by block
subspace iteration followed by a Rayleigh-Ritz step.  Each mode is zero
outside the pupil, has zero mean over it and unit RMS (1 nm) over it, and
modes are mutually orthogonal over the pupil.

The basis must not depend on the machine's linear-algebra rounding, so that
results computed with it on one machine (stored expected values) refer to
the same modes on another.  The square pixel grid gives the circular pupil
the symmetries of the square, under which many eigenvalues are exactly
degenerate in pairs; an eigen-solver returns an arbitrary orthonormal basis
of such a pair's plane, chosen by rounding (and the subspace iteration,
stopped before the tail is converged, splits such pairs by up to ~1e-6, so
a rotation inside them is as ill-determined).  So the Ritz vectors are
grouped into clusters of nearly equal Ritz values (relative gap below 1e-4;
a cluster may then join two distinct modes, which only mixes two columns
of the basis inside their common span), and
each cluster's basis is replaced by a canonical one: the orthonormal basis
of the same subspace whose inner products with the first seeded Gaussian
probe fields form a lower-triangular matrix with a positive diagonal
(Gram-Schmidt on the probes' projections).  This fixes every mode's
direction, including its sign, before the leading modes are kept.
"""
from __future__ import annotations

import hashlib
import os

import numpy as np
import scipy.fft as sfft
from scipy.special import gamma, kv

_WORKERS = os.cpu_count() or 1


def _cov_kernel(P: int, pixel_m: float, L0_m: float) -> np.ndarray:
    n = 2 * P
    d = np.arange(n)
    d = np.where(d < P, d, d - n).astype(np.float64)        # signed offsets
    r = np.hypot(d[:, None], d[None, :]) * pixel_m
    x = 2 * np.pi * r / L0_m
    with np.errstate(invalid="ignore"):
        c = x ** (5.0 / 6.0) * kv(5.0 / 6.0, x)
    c[r == 0] = 2.0 ** (-1.0 / 6.0) * gamma(5.0 / 6.0)
    return sfft.rfft2(c)


def probe_fields(npix: int, m: int) -> np.ndarray:
    """[npix, m] seeded Gaussian fields over the pupil pixels that fix the
    modes' directions within degenerate clusters."""
    return np.random.default_rng(20161607).standard_normal((m, npix)).T


def _canonical_clusters(w: np.ndarray, V: np.ndarray, X: np.ndarray, rel_gap: float = 1e-4) -> np.ndarray:
    """Eigenvectors V (columns, eigenvalues w descending) with each cluster of
    equal eigenvalues rotated to the canonical basis of its subspace: the
    Ritz vectors U = X V of a cluster of size c are replaced by the
    orthonormal basis Q of span(U) with probe_j . Q_i = 0 for j < i and
    probe_i . Q_i > 0 (i, j < c)."""
    V = V.copy()
    n = len(w)
    i = 0
    while i < n:
        j = i + 1
        while j < n and abs(w[j - 1] - w[j]) <= rel_gap * abs(w[i]):
            j += 1
        c = j - i
        W = probe_fields(X.shape[0], c)
        G = (W.T @ X) @ V[:, i:j]                # [c probes, c vectors]
        # rotation R with G R lower-triangular, positive diagonal: from the QR
        # factors of G^T (G^T = Q T, so G Q = T^T is lower-triangular)
        Q, T = np.linalg.qr(G.T)
        Q = Q * np.where(np.diag(T) < 0.0, -1.0, 1.0)[None, :]
        V[:, i:j] = V[:, i:j] @ Q
        i = j
    return V


def kl_modes(A: np.ndarray, pixel_m: float, L0_m: float, n_modes: int,
             iters: int = 8, oversample: int = 64, seed: int = 12345,
             cache: bool = True) -> np.ndarray:
    """[n_modes, P, P] float64 KL modes (unit RMS in nm over the pupil)."""
    P = A.shape[0]
    key = hashlib.sha1(np.packbits(A.astype(bool)).tobytes()
                       + repr((P, pixel_m, L0_m, n_modes, iters, oversample, seed,
                               "canonical-v2")).encode()).hexdigest()[:16]
    cdir = os.environ.get("PWFS_CACHE_DIR", os.path.join(os.path.expanduser("~"), ".cache", "pwfs_kl"))
    path = os.path.join(cdir, f"kl_{key}.npy")
    if cache and os.path.exists(path):
        return np.load(path)
    pix = np.flatnonzero(A.ravel() > 0)
    npix = pix.size
    Ck = _cov_kernel(P, pixel_m, L0_m)

    def apply(X):                               # X [npix, m] -> Q C Q X
        X = X - X.mean(axis=0, keepdims=True)
        m = X.shape[1]
        out = np.empty_like(X)
        step = 128
        for s in range(0, m, step):
            blk = X[:, s:s + step]
            flat = np.zeros((blk.shape[1], P * P))
            flat[:, pix] = blk.T
            g = np.zeros((blk.shape[1], 2 * P, 2 * P))
            g[:, :P, :P] = flat.reshape(-1, P, P)
            y = sfft.irfft2(sfft.rfft2(g, workers=_WORKERS) * Ck, s=(2 * P, 2 * P), workers=_WORKERS)
            out[:, s:s + step] = y[:, :P, :P].reshape(blk.shape[1], -1)[:, pix].T
        return out - out.mean(axis=0, keepdims=True)

    rng = np.random.default_rng(seed)
    m = min(n_modes + oversample, npix - 1)
    X = np.linalg.qr(apply(rng.standard_normal((npix, m))))[0]
    for _ in range(iters):
        X = np.linalg.qr(apply(X))[0]
    H = X.T @ apply(X)
    w, V = np.linalg.eigh(0.5 * (H + H.T))
    order = np.argsort(w)[::-1]
    w, V = w[order], _canonical_clusters(w[order], V[:, order], X)
    U = X @ V[:, :n_modes]                       # orthonormal columns, piston-free
    U -= U.mean(axis=0, keepdims=True)           # (to rounding: exactly zero mean)
    modes = np.zeros((n_modes, P * P))
    modes[:, pix] = U.T * np.sqrt(npix)
    modes = modes.reshape(n_modes, P, P)
    if cache:
        os.makedirs(cdir, exist_ok=True)
        tmp = path + f".{os.getpid()}.tmp.npy"
        np.save(tmp, modes)
        os.replace(tmp, path)
    return modes
