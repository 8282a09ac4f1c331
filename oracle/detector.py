"""FP64 reference of the detector step (the paper's CCD object, Sec. 4 and
Tab. 1 "ccd": it integrates the pupil-plane intensity into pixels with photon
noise, readout noise and a quantum efficiency).

Test infrastructure only (see the package docstring).

Model (readings; the paper gives the parameters, not the algorithm):
  * mean photo-electrons of a pixel: lam = g * I, with I the noiseless binned
    pupil intensity and g (float32) electrons per unit intensity, chosen by
    the caller so that a flat wavefront collects the frame's photo-electron
    budget (flux x band x area x exposure x QE);
  * photon noise: k ~ Poisson(lam);  readout noise: + ron * z, z ~ N(0, 1);
    the pixel value is k + ron z (float32, electrons).
Random numbers come from the counter-based generator Philox4x32-10
(Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2,
3", SC'11), key = the 64-bit seed (low word first), counter =
(pixel index j, frame index low word, frame index high word, draw word d),
each call giving four 32-bit words; a word x maps to the uniform
u = (x + 1/2) 2^-32 in (0, 1).  The Poisson count uses the draw words
d = 0, 1, 2, ... (four uniforms each) in order; the readout noise uses
d = 2^31 (its first two uniforms), so it does not depend on how many
uniforms the count consumed.
Poisson count (exact, by multiplying uniforms, in FP64): lam is split into
n = ceil(lam / 500) equal pieces; for each piece, with L = exp(-lam / n),
the number of uniforms whose running product stays above L before it falls
to L or below.  Above lam = 1e4 the count is the normal approximation
floor(lam + sqrt(lam) z' + 1/2), clipped at 0, with z' from the second pair
of the readout-noise draw (d = 2^31, uniforms 2 and 3).
Box-Muller: z = sqrt(-2 ln u1) cos(2 pi u2), z' = sqrt(-2 ln u3) cos(2 pi u4).
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57          # Philox4x32 multipliers
W0, W1 = 0x9E3779B9, 0xBB67AE85          # Weyl key increments
PIECE = 500.0
NORMAL_ABOVE = 1.0e4
RON_WORD = 1 << 31
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten rounds of Philox4x32 on arrays of counters (uint32 values in any
    integer dtype); returns four uint64 arrays holding 32-bit words."""
    c = [np.asarray(x, np.uint64) & _MASK for x in (c0, c1, c2, c3)]
    c = [np.broadcast_to(x, np.broadcast(*c).shape).copy() for x in c]
    k0 = np.uint64(int(k0) & 0xFFFFFFFF)
    k1 = np.uint64(int(k1) & 0xFFFFFFFF)
    for _ in range(10):
        p0 = np.uint64(M0) * c[0]
        p1 = np.uint64(M1) * c[2]
        c = [((p1 >> np.uint64(32)) ^ c[1] ^ k0) & _MASK, p1 & _MASK,
             ((p0 >> np.uint64(32)) ^ c[3] ^ k1) & _MASK, p0 & _MASK]
        k0 = (k0 + np.uint64(W0)) & _MASK
        k1 = (k1 + np.uint64(W1)) & _MASK
    return c


def uniform(x):
    """(x + 1/2) 2^-32 in FP64, x a 32-bit word: strictly inside (0, 1)."""
    return (np.asarray(x, np.float64) + 0.5) * 2.0 ** -32


def _words(j, frame, d, seed):
    f = int(frame)
    return philox4x32_10(j, f & 0xFFFFFFFF, f >> 32, d, seed & 0xFFFFFFFF, seed >> 32)


def poisson_counts(lam, frame: int, seed: int):
    """Photon counts of the pixels j = 0..len(lam)-1 of one frame (int64)."""
    lam = np.asarray(lam, np.float64)
    n = lam.size
    j = np.arange(n, dtype=np.uint64)
    out = np.zeros(n, np.int64)
    ron = _words(j, frame, RON_WORD, seed)
    u3, u4 = uniform(ron[2]), uniform(ron[3])
    big = lam > NORMAL_ABOVE
    if big.any():
        z2 = np.sqrt(-2.0 * np.log(u3[big])) * np.cos(2.0 * np.pi * u4[big])
        out[big] = np.maximum(0.0, np.floor(lam[big] + np.sqrt(lam[big]) * z2 + 0.5)).astype(np.int64)
    idx = np.nonzero((lam > 0.0) & ~big)[0]
    if idx.size == 0:
        return out
    npieces = np.ceil(lam[idx] / PIECE)
    L = np.exp(-(lam[idx] / npieces))
    piece = np.zeros(idx.size)            # pieces finished
    p = np.ones(idx.size)
    k = np.zeros(idx.size, np.int64)
    t = 0                                  # uniforms consumed so far (same for every active pixel)
    active = np.ones(idx.size, bool)
    while active.any():
        a = np.nonzero(active)[0]
        w = _words(j[idx[a]], frame, t >> 2, seed)[t & 3]
        u = uniform(w)
        p[a] = p[a] * u
        done = p[a] <= L[a]
        k[a[~done]] += 1
        fin = a[done]
        piece[fin] += 1
        p[fin] = 1.0
        active[fin[piece[fin] >= npieces[fin]]] = False
        t += 1
    out[idx] = k
    return out


def gaussians(n: int, frame: int, seed: int):
    """Readout-noise deviates z of the pixels j = 0..n-1 of one frame."""
    w = _words(np.arange(n, dtype=np.uint64), frame, RON_WORD, seed)
    u1, u2 = uniform(w[0]), uniform(w[1])
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def detect(intensity, gain: float, ron_e: float, seed: int, frame0: int):
    """Detector pixels [B, ...] (float32 electrons) from noiseless intensity
    [B, ...]; frame b uses frame index frame0 + b."""
    I = np.asarray(intensity, np.float32)
    B = I.shape[0]
    g = np.float64(np.float32(gain))
    out = np.empty(I.shape, np.float32)
    for b in range(B):
        lam = g * I[b].ravel().astype(np.float64)
        k = poisson_counts(lam, frame0 + b, seed)
        z = gaussians(lam.size, frame0 + b, seed)
        out[b] = (k + float(ron_e) * z).astype(np.float32).reshape(I.shape[1:])
    return out
