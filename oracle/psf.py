"""FP64 reference of the PSF camera (the paper's PSF object, Sec. 4 and
Tab. 1 "psf": the point-spread function of the residual wavefront at a
science wavelength, with a padding factor, its Strehl ratio and its
integration over the run).

Test infrastructure only (see the package docstring).

Definition (literal): the pupil field E = A exp(i phi), phi = 2 pi opd[nm]
1e-9 / lambda, is zero-padded to N = pad * P and
    PSF[v, u] = |FFT2(E)[v - N/2, u - N/2]|^2 / (sum A)^2
(unnormalised forward transform, frequency index taken modulo N, zero
frequency at (N/2, N/2)), so a flat wavefront peaks at exactly 1 there and
the value at (N/2, N/2) is the Strehl ratio |sum A exp(i phi)|^2 / (sum A)^2.
One lambda/D is `pad` pixels.  The integrated (long-exposure) PSF is the sum
of the frames' PSFs.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft

_WORKERS = int(os.environ.get("ORACLE_FFT_WORKERS", os.cpu_count() or 1))


def field(opd_nm, amp, wavelength_m):
    phi = 2.0 * np.pi * np.asarray(opd_nm, np.float64) * 1e-9 / wavelength_m
    return np.asarray(amp, np.float64) * np.exp(1j * phi)


def psf(opd_nm, amp, wavelength_m: float, pad: int):
    """PSF [N, N] of one frame (opd [P, P] in nm)."""
    A = np.asarray(amp, np.float64)
    P = A.shape[0]
    N = pad * P
    E = np.zeros((N, N), np.complex128)
    E[:P, :P] = field(opd_nm, A, wavelength_m)
    F = scipy.fft.fft2(E, workers=_WORKERS)
    return np.fft.fftshift(np.abs(F) ** 2) / A.sum() ** 2


def strehl(opd_nm, amp, wavelength_m: float):
    A = np.asarray(amp, np.float64)
    return float(np.abs(field(opd_nm, A, wavelength_m).sum()) ** 2 / A.sum() ** 2)
