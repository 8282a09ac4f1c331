"""Seeded von Karman phase screens (input generation, host FP64).

Screens are drawn with the FFT method: complex white noise shaped by the
square root of the von Karman phase power spectrum
    W(f) = 0.023 r0^(-5/3) (f^2 + L0^-2)^(-11/6)   [rad^2 m^2 at r0's wavelength]
and summed over the discrete frequency grid.  The piston term is set to
zero.  The result is returned as optical path difference in nanometres
(phase * lambda_r0 / 2 pi), stored as float32 because that is the input
precision of the sensor.
"""
from __future__ import annotations

import numpy as np

from .configs import AtmoConfig, SensorConfig


def von_karman_opd_nm(n: int, pixel_m: float, r0_m: float, L0_m: float,
                      rng: np.random.Generator,
                      r0_wavelength_m: float = 500e-9) -> np.ndarray:
    """One n x n screen in nm OPD (float64)."""
    f = np.fft.fftfreq(n, d=pixel_m)
    f2 = f[:, None] ** 2 + f[None, :] ** 2
    psd = 0.023 * r0_m ** (-5.0 / 3.0) * (f2 + 1.0 / L0_m ** 2) ** (-11.0 / 6.0)
    psd[0, 0] = 0.0
    df = 1.0 / (n * pixel_m)
    noise = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    phase = np.real(np.fft.fft2(np.sqrt(psd) * df * noise))
    return phase * (r0_wavelength_m / (2.0 * np.pi)) * 1e9


def screen_size_for(cfg: SensorConfig, L0_m: float, minimum: int = 0) -> int:
    """Smallest power of two covering both the pupil and one outer scale."""
    need = max(cfg.n_pupil, int(np.ceil(L0_m / cfg.pixel_m)), minimum)
    return 1 << int(np.ceil(np.log2(need)))


def open_loop_batch(cfg: SensorConfig, atmo: AtmoConfig, seeds, r0_range=None,
                    screen_n: int | None = None) -> tuple[np.ndarray, np.ndarray]:
    """Independent P x P screens, one per seed (centre crop of a larger screen).

    Returns (opd [B, P, P] float32 nm, r0 [B] float64).  With r0_range the
    Fried parameter of each screen is drawn uniformly from that interval
    using the same seed.
    """
    P = cfg.n_pupil
    n = screen_n or screen_size_for(cfg, atmo.L0_m)
    out = np.empty((len(seeds), P, P), np.float32)
    r0s = np.empty(len(seeds))
    for i, s in enumerate(seeds):
        rng = np.random.default_rng(int(s))
        r0 = atmo.r0_m if r0_range is None else rng.uniform(*r0_range)
        scr = von_karman_opd_nm(n, cfg.pixel_m, r0, atmo.L0_m, rng, atmo.r0_wavelength_m)
        o = (n - P) // 2
        out[i] = scr[o:o + P, o:o + P]
        r0s[i] = r0
    return out, r0s


def frozen_flow_sequence(cfg: SensorConfig, atmo: AtmoConfig, n_steps: int, seed: int,
                         screen_n: int = 2048) -> np.ndarray:
    """Single-layer frozen flow: a large screen translated along +x.

    Frame t samples the screen at x = x0 - t * v / (rate * pixel) + j with
    bilinear interpolation (only the x coordinate is fractional), so the
    turbulence pattern moves toward +x at the wind speed.  Returns
    [n_steps, P, P] float32 nm.
    """
    P = cfg.n_pupil
    rng = np.random.default_rng(int(seed))
    scr = von_karman_opd_nm(screen_n, cfg.pixel_m, atmo.r0_m, atmo.L0_m, rng,
                            atmo.r0_wavelength_m)
    step_px = atmo.wind_m_s / (atmo.frame_rate_hz * cfg.pixel_m)
    span = step_px * (n_steps - 1)
    if span + P + 2 > screen_n:
        raise ValueError("screen too small for the requested sequence")
    y0 = (screen_n - P) // 2
    x0 = int(np.ceil(span)) + (screen_n - P - int(np.ceil(span)) - 1) // 2
    rows = scr[y0:y0 + P]
    out = np.empty((n_steps, P, P), np.float32)
    j = np.arange(P)
    for t in range(n_steps):
        xs = x0 - t * step_px + j
        xi = np.floor(xs).astype(np.int64)
        w = xs - xi
        out[t] = (1.0 - w) * rows[:, xi] + w * rows[:, xi + 1]
    return out


def cfg4_loop_sequence(cfg: SensorConfig, atmo: AtmoConfig, seed: int, n_steps: int,
                       r0_range=(0.08, 0.2)) -> tuple[np.ndarray, float]:
    """Frozen-flow sequence of one precision-study loop: r0 is the first
    uniform draw of default_rng(seed) in r0_range (the r0 of that seed's
    open-loop screen), the screen and its motion those of
    frozen_flow_sequence with seed 10000 + seed.  Returns (seq, r0)."""
    r0 = float(np.random.default_rng(int(seed)).uniform(*r0_range))
    at = AtmoConfig(r0_m=r0, L0_m=atmo.L0_m, r0_wavelength_m=atmo.r0_wavelength_m,
                    wind_m_s=atmo.wind_m_s, frame_rate_hz=atmo.frame_rate_hz)
    return frozen_flow_sequence(cfg, at, n_steps, seed=10000 + int(seed)), r0


def tilt_opd_nm(P: int, alpha_lod: float, wavelength_m: float, axis: str = "x") -> np.ndarray:
    """Pure tilt of alpha lambda/D across the pupil: phase 2 pi alpha x / P.

    x is the pixel index measured from the pupil centre (P-1)/2; returned in
    nm at the given wavelength (float64).
    """
    c = (P - 1) / 2.0
    x = np.arange(P) - c
    ramp = np.broadcast_to(x[None, :] if axis == "x" else x[:, None], (P, P))
    return alpha_lod * ramp / P * wavelength_m * 1e9


class CropBank:
    """Random P x P crops of a few large von Karman screens (input generation).

    For a fixed outer scale the von Karman phase PSD scales as r0^(-5/3), so
    a screen drawn at r0_ref becomes a screen at r0 when multiplied by
    (r0_ref / r0)^(5/6); each crop also gets one of the 8 square symmetries.
    Crops of one screen overlap, which is acceptable for training inputs.
    """

    def __init__(self, cfg: SensorConfig, L0_m: float, n_screens: int, screen_n: int, seed: int,
                 r0_ref_m: float = 0.1):
        self.P = cfg.n_pupil
        self.r0_ref = r0_ref_m
        rng = np.random.default_rng(int(seed))
        self.screens = [von_karman_opd_nm(screen_n, cfg.pixel_m, r0_ref_m, L0_m, rng).astype(np.float32)
                        for _ in range(n_screens)]

    def draw(self, rng: np.random.Generator, n: int, r0_range) -> tuple[np.ndarray, np.ndarray]:
        """(opd [n, P, P] float32 nm, r0 [n])."""
        P = self.P
        out = np.empty((n, P, P), np.float32)
        r0 = rng.uniform(*r0_range, size=n)
        for i in range(n):
            s = self.screens[rng.integers(len(self.screens))]
            y, x = rng.integers(0, s.shape[0] - P, size=2)
            c = s[y:y + P, x:x + P]
            sym = rng.integers(8)
            if sym & 1:
                c = c[::-1]
            if sym & 2:
                c = c[:, ::-1]
            if sym & 4:
                c = c.T
            out[i] = c * np.float32((self.r0_ref / r0[i]) ** (5.0 / 6.0))
        return out, r0


def layered_opd_nm(cfg: SensorConfig, atmo: AtmoConfig, layers, directions_arcsec, seed: int,
                   screen_n: int = 1024) -> np.ndarray:
    """OPD seen by several guide stars through a layered atmosphere.

    layers: (altitude m, Cn2 fraction) pairs; each layer is a von Karman
    screen with r0_layer = r0 * fraction^(-3/5) (so the fractions add up in
    r0^(-5/3)).  A star at angle (tx, ty) sees layer h shifted by h * (tx, ty)
    (natural guide stars, no cone effect); the shift is applied by bilinear
    interpolation in FP64.  Returns [n_dir, P, P] float32 nm."""
    P = cfg.n_pupil
    rng = np.random.default_rng(int(seed))
    arcsec = np.pi / (180.0 * 3600.0)
    out = np.zeros((len(directions_arcsec), P, P))
    for h, frac in layers:
        r0 = atmo.r0_m * float(frac) ** (-3.0 / 5.0)
        scr = von_karman_opd_nm(screen_n, cfg.pixel_m, r0, atmo.L0_m, rng, atmo.r0_wavelength_m)
        for i, (tx, ty) in enumerate(directions_arcsec):
            sx = h * tx * arcsec / cfg.pixel_m
            sy = h * ty * arcsec / cfg.pixel_m
            x0 = (screen_n - P) / 2.0 + sx
            y0 = (screen_n - P) / 2.0 + sy
            ix, iy = int(np.floor(x0)), int(np.floor(y0))
            fx, fy = x0 - ix, y0 - iy
            if ix < 0 or iy < 0 or ix + P + 1 > screen_n or iy + P + 1 > screen_n:
                raise ValueError("screen too small for the guide-star separation")
            blk = scr[iy:iy + P + 1, ix:ix + P + 1]
            out[i] += ((1 - fy) * ((1 - fx) * blk[:-1, :-1] + fx * blk[:-1, 1:])
                       + fy * ((1 - fx) * blk[1:, :-1] + fx * blk[1:, 1:]))
    return out.astype(np.float32)
