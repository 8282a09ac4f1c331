"""FP64 reference of the Shack-Hartmann sensor (the paper's second sensor
type, Sec. 1 and Sec. 6; the paper gives no parameters, so the geometry is a
reading: n_sub x n_sub square subapertures of s = P / n_sub pupil pixels).

Test infrastructure only (see the package docstring).

Definition (literal): for subaperture (iy, ix) the field
E = A exp(i phi) over its s x s pixels, phi = 2 pi opd[nm] 1e-9 / lambda, is
zero-padded to M = pad s and
    spot[v, u] = |FFT2(E)[v - M/2, u - M/2]|^2      (u, v = 0 .. M-1)
(unnormalised forward transform, indices modulo M, zero frequency at
(M/2, M/2); one spot pixel is lambda / (pad d), d the subaperture size).
Centroid (centre of gravity over the whole M x M box):
    cx = sum spot (u - M/2) / sum spot,   cy likewise with v.
Valid subapertures: pupil fill fraction >= 0.5 (the sensor's rule).
Slopes [cx over V ; cy over V] in spot pixels, minus those of a flat
wavefront.
"""
from __future__ import annotations

import numpy as np

from .pwfs import pupil_amplitude, valid_subapertures


class ShackHartmann:
    def __init__(self, n_pupil: int, n_sub: int, pad: int, wavelength_m: float, obstruction: float = 0.0,
                 amp=None):
        self.P, self.n_sub, self.pad = n_pupil, n_sub, pad
        self.s = n_pupil // n_sub
        self.M = pad * self.s
        self.lam = wavelength_m
        self.A = pupil_amplitude(n_pupil, obstruction) if amp is None else np.asarray(amp, np.float64)
        self.valid = valid_subapertures(self.A, self.s)
        self.n_valid = self.valid.size
        self.ref = np.zeros(2 * self.n_valid)
        self.ref = self._raw(np.zeros((n_pupil, n_pupil)))[1]

    def spots(self, opd_nm):
        """Spots [n_valid, M, M] of one frame."""
        s, M, S = self.s, self.M, self.n_sub
        E = self.A * np.exp(2j * np.pi * np.asarray(opd_nm, np.float64) * 1e-9 / self.lam)
        sub = E.reshape(S, s, S, s).transpose(0, 2, 1, 3).reshape(S * S, s, s)[self.valid]
        pad = np.zeros((sub.shape[0], M, M), np.complex128)
        pad[:, :s, :s] = sub
        F = np.fft.fft2(pad, axes=(1, 2))
        return np.fft.fftshift(np.abs(F) ** 2, axes=(1, 2))

    def _raw(self, opd_nm):
        sp = self.spots(opd_nm)
        M = self.M
        c = np.arange(M) - M // 2
        tot = sp.sum(axis=(1, 2))
        cx = (sp * c[None, None, :]).sum(axis=(1, 2)) / tot
        cy = (sp * c[None, :, None]).sum(axis=(1, 2)) / tot
        return sp, np.concatenate([cx, cy]) - self.ref

    def measure(self, opd_nm):
        """(spots [n_valid, M, M], slopes [2 n_valid]) of one frame."""
        return self._raw(opd_nm)
