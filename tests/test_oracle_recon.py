"""Pins of the oracle's calibration, reconstructor and integrator loop."""
import numpy as np
import pytest

from synth.configs import SensorConfig
from synth.kl import kl_modes
import oracle
from oracle import recon


def _linear_world(P=8, M=5, ns=14, seed=0):
    rng = np.random.default_rng(seed)
    A = np.ones((P, P))
    Q, _ = np.linalg.qr(rng.standard_normal((P * P, M + 1)))
    Q = Q[:, 1:] - Q[:, 1:].mean(axis=0)                  # piston-free
    Q, _ = np.linalg.qr(Q)
    modes = (Q.T * np.sqrt(P * P)).reshape(M, P, P)       # unit RMS, orthogonal
    G = rng.standard_normal((ns, M))

    def measure(r):
        coeff = modes.reshape(M, -1) @ np.asarray(r).ravel() / (P * P)
        return G @ coeff
    return A, modes, G, measure


def test_push_pull_im_and_pinv_on_linear_sensor():
    A, modes, G, measure = _linear_world()
    IM = recon.interaction_matrix(measure, modes, 10.0)
    assert np.abs(IM - G).max() < 1e-12
    R, sig = recon.pseudo_inverse(IM)
    assert np.abs(R @ IM - np.eye(IM.shape[1])).max() < 1e-12
    assert np.allclose(sig, np.linalg.svd(G, compute_uv=False))


def test_integrator_delay_two_recursion():
    """Static disturbance, exact sensor: the modal residual obeys
    e(t) = e(t-1) - g e(t-2) with e(0) = e(1) = a (delay 2)."""
    A, modes, G, measure = _linear_world()
    R, _ = recon.pseudo_inverse(G)
    a = np.array([30.0, -12.0, 5.0, 0.0, 7.0])
    atm = np.tensordot(a, modes, axes=1)
    T, g = 25, 0.4
    rms, c = recon.closed_loop(measure, np.repeat(atm[None], T, 0), modes, R, g, 2, A)
    e = [a, a]
    for t in range(2, T):
        e.append(e[-1] - g * e[-2])
    e = np.array(e)
    assert np.abs(rms - np.linalg.norm(e, axis=1)).max() < 1e-9
    assert np.abs(c[0] - g * a).max() < 1e-12 and np.abs(c[1] - 2 * g * a).max() < 1e-12
    # Gain 0.4 at delay 2 is stable: the residual decays.
    assert rms[-1] < 0.05 * rms[0]


def test_loop_residual_metric_settle():
    assert recon.loop_residual_nm(np.array([100.0, 100.0, 3.0, 4.0]), 2) == pytest.approx(np.sqrt(12.5))
    A = np.ones((4, 4))
    assert recon.residual_rms_nm(np.full((4, 4), 7.0), A) == 0.0


SMALL = SensorConfig(name="small", n_fft=64, n_pupil=16, n_bin=2, n_mod=8,
                     mod_radius_lod=3.0, wavelength_m=750e-9, diameter_m=2.0)


def test_pwfs_reconstructor_recovers_single_modes():
    orc = oracle.Oracle(SMALL)
    modes = kl_modes(orc.A, SMALL.pixel_m, 20.0, 20, cache=False)
    meas = lambda r: orc.measure(r)[1]
    IM = recon.interaction_matrix(meas, modes, 10.0)
    R, sig = recon.pseudo_inverse(IM)
    assert np.abs(R @ IM - np.eye(20)).max() < 1e-10
    for i in (0, 5, 19):
        m = R @ meas(5.0 * modes[i])
        exp = np.zeros(20); exp[i] = 5.0
        assert np.abs(m - exp).max() < 0.05 * 5.0
