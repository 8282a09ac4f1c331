"""Sensor and atmosphere configurations of the modulated pyramid workloads.

Plain records: both the oracle and the HIP path read the same numbers,
neither shares code with the other through this module.

Parameter provenance.  The paper's example (Sec. 4, Tab. 1, "pyramid",
"detector", "atmo" and "control" blocks) fixes the kind of system: an 8 m
class pupil, a modulated four-face pyramid at 750 nm with a modulation
radius of 3 lambda/D, a 1 ms step and an integrator with a delay of two
steps.  The sizes below are the measured workloads; the conventions the paper
leaves open (pupil centring, mask apex, face shift, modulation phase
origin, normalisation, ...) are applied identically by both
implementations.
"""
from __future__ import annotations

from dataclasses import dataclass, replace, asdict

import numpy as np


@dataclass(frozen=True)
class SensorConfig:
    """Geometry of one modulated pyramid sensor.

    n_fft       N: side of the square FFT grid (pupil plane == focal plane grid).
    n_pupil     P: pupil diameter in pupil-plane pixels.
    n_bin       b: detector binning; S = P / b subapertures across.
    det_window  S > 0: instead of binning, each P-pixel pupil window is
                resampled to S detector pixels of pitch P / S (non-integer
                rebin; needs n_bin 1); S subapertures across.
    field_stop_lod  diameter of a circular focal-plane field stop in the
                units of mod_radius_lod (0: none).
    n_mod       K: modulation points on the circle.
    face_shift  Delta: pupil-image displacement in pixels produced by each
                pyramid face; 0 selects N / 4.
    norm_mode   0: slopes divided by the mean total flux over valid
                subapertures of the current frame; 1: by each
                subaperture's own total flux.
    mod_radius_lod  modulation radius in lambda / D.
    wavelength_m    sensing wavelength.
    diameter_m      telescope diameter (sets the metric pixel size P / D).
    obstruction     central obstruction as a fraction of the diameter.
    """
    name: str
    n_fft: int
    n_pupil: int
    n_bin: int
    n_mod: int
    mod_radius_lod: float
    wavelength_m: float
    diameter_m: float
    obstruction: float = 0.0
    face_shift: int = 0
    norm_mode: int = 0
    det_window: int = 0
    field_stop_lod: float = 0.0

    @property
    def n_sub(self) -> int:
        return self.det_window if self.det_window else self.n_pupil // self.n_bin

    @property
    def delta(self) -> int:
        return self.face_shift if self.face_shift else self.n_fft // 4

    @property
    def pixel_m(self) -> float:
        return self.diameter_m / self.n_pupil

    def with_(self, **kw) -> "SensorConfig":
        return replace(self, **kw)

    def as_dict(self) -> dict:
        return asdict(self)


@dataclass(frozen=True)
class AtmoConfig:
    """Von Karman turbulence used to draw the input phase screens.

    r0_m is quoted at r0_wavelength_m (500 nm); screens are returned as
    optical path difference in nanometres, which is achromatic.
    """
    r0_m: float
    L0_m: float
    r0_wavelength_m: float = 500e-9
    wind_m_s: float = 0.0
    frame_rate_hz: float = 1000.0


# Plain single-source sensor: 8 m pupil on 32 px, 128-point FFT grid,
# 16 modulation points on a 3 lambda/D ring at 750 nm, pupils separated
# by 64 px (Delta = 32), 2x2 binning to 16x16 subapertures.
CFG1 = SensorConfig(name="cfg1_n128_p32_k16", n_fft=128, n_pupil=32, n_bin=2,
                    n_mod=16, mod_radius_lod=3.0, wavelength_m=750e-9,
                    diameter_m=8.0)
ATMO1 = AtmoConfig(r0_m=0.15, L0_m=25.0)

# LBT-like SCAO sensor: 8.4 m pupil on 160 px, 640-point FFT grid,
# 48 modulation points at 3 lambda/D, 750 nm, 40x40 subapertures.
CFG2 = SensorConfig(name="cfg2_n640_p160_k48", n_fft=640, n_pupil=160, n_bin=4,
                    n_mod=48, mod_radius_lod=3.0, wavelength_m=750e-9,
                    diameter_m=8.4)
ATMO2 = AtmoConfig(r0_m=0.12, L0_m=40.0, wind_m_s=15.0, frame_rate_hz=1000.0)

# The paper's detector geometry (Tab. 1 "pyramid": output_resolution 80,
# pupils pup_diam 30 pixels across with centres pup_dist 36 apart; 3 lambda/D
# modulation at 750 nm).  Each P = 160 pupil window is resampled to 36
# detector pixels (pitch 4.44 pupil pixels); the window spans 36 / 30 pupil
# diameters, so the pupil is 133.3 pixels across (paper_pupil) and the
# window-relative diameter and modulation radius carry that factor.
PAPER_PUP_DIAM, PAPER_PUP_DIST, PAPER_DET_PX = 30, 36, 80
CFG_PAPER_DET = SensorConfig(name="paper_det80_n640_p160_k48", n_fft=640, n_pupil=160, n_bin=1,
                             n_mod=48, mod_radius_lod=3.0 * 36 / 30, wavelength_m=750e-9,
                             diameter_m=8.4 * 36 / 30, det_window=36)


def paper_pupil(P: int, pup_diam: int = PAPER_PUP_DIAM, pup_dist: int = PAPER_PUP_DIST):
    """Binary circular pupil of diameter P pup_diam / pup_dist pixels centred
    in the P x P window (float32)."""
    import numpy as np
    c = (P - 1) / 2.0
    y, x = np.mgrid[0:P, 0:P]
    r = P * pup_diam / pup_dist / 2.0
    return (((x - c) ** 2 + (y - c) ** 2) <= r * r).astype(np.float32)


# Precision study on the same shapes: 16 independent screens with
# r0 drawn uniformly in [0.08, 0.2] m (L0 as in the closed loop).
CFG4_R0_RANGE = (0.08, 0.2)
CFG4_SEEDS = tuple(range(16))
# Closed loops of the precision study: frozen-flow sequences whose r0 is the
# one drawn for the same seed's open-loop screen (first draw of the seed's
# generator), 500 steps each; the sequence itself uses seed 10000 + seed.
CFG4_LOOP_SEEDS = (0, 1, 2, 3, 4, 5)
CFG4_LOOP_STEPS = 500
# The LBT-like loop of the benchmark: r0 0.12 m, 1000 steps, sequence seed.
CFG2_LOOP_SEED = 2024
CFG2_LOOP_STEPS = 1000

# 40 m class multi-source sensor: six guide stars on a 45 arcsec ring seen
# through a three-layer atmosphere, sensed at 650 and 850 nm.  The
# modulation mirror's angular amplitude is fixed, so the radius is 3 lambda/D
# at 650 nm and 3 * 650/850 lambda/D at 850 nm.
CFG3 = SensorConfig(name="cfg3_n1920_p480_k64", n_fft=1920, n_pupil=480, n_bin=5,
                    n_mod=64, mod_radius_lod=3.0, wavelength_m=650e-9,
                    diameter_m=39.0)
CFG3_850 = SensorConfig(name="cfg3_n1920_p480_k64_850nm", n_fft=1920, n_pupil=480, n_bin=5,
                        n_mod=64, mod_radius_lod=3.0 * 650.0 / 850.0, wavelength_m=850e-9,
                        diameter_m=39.0)
ATMO3 = AtmoConfig(r0_m=0.15, L0_m=25.0)
CFG3_LAYERS = ((0.0, 0.6), (5000.0, 0.25), (12000.0, 0.15))       # (altitude m, Cn2 fraction)
CFG3_GS_ARCSEC = tuple((45.0 * float(np.cos(2 * np.pi * i / 6)), 45.0 * float(np.sin(2 * np.pi * i / 6)))
                       for i in range(6))

# Closed-loop constants of the integrator (gain of the LBT-like loop,
# delay of the paper's example control block).
LOOP_GAIN = 0.4
LOOP_DELAY = 2
LOOP_SETTLE_STEPS = 50
N_KL_MODES = 600
PUSH_PULL_NM = 10.0

CONFIGS = {"cfg1": CFG1, "cfg2": CFG2, "cfg3": CFG3}


# Photon budget of the paper's example detector: magnitude-8 source, 300 nm
# band, QE 0.32, 1 ms exposure, readout noise 1 e-.  Zero point: 3.9e7
# photons / s / m^2 / nm at magnitude 0 (a magnitude-0 star near 700 nm).
ZERO_POINT_PH_S_M2_NM = 3.9e7
DETECTOR_MAG = 8.0
DETECTOR_BAND_NM = 300.0
DETECTOR_QE = 0.32
DETECTOR_RON_E = 1.0


def photoelectrons_per_frame(cfg: SensorConfig, magnitude: float = DETECTOR_MAG, band_nm: float = DETECTOR_BAND_NM,
                             qe: float = DETECTOR_QE, exposure_s: float = 1e-3,
                             zero_point: float = ZERO_POINT_PH_S_M2_NM) -> float:
    """Photo-electrons collected by the pupil in one exposure."""
    area = np.pi * (cfg.diameter_m / 2.0) ** 2 * (1.0 - cfg.obstruction ** 2)
    return zero_point * 10.0 ** (-0.4 * magnitude) * band_nm * area * exposure_s * qe
