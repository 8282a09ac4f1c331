"""Pins of the FP64 CNN oracle: brute-force convolution, finite-difference
gradients, Adam's closed form, input normalisation and modal projection."""
import numpy as np
import pytest

from oracle import cnn
from synth.kl import kl_modes
from oracle.pwfs import pupil_amplitude


def _rand_params(shapes, rng, scale=None):
    """Normal weights; scale None = He scaling sqrt(2 / fan_in) (keeps activations O(1))."""
    out = {}
    for k, s in shapes.items():
        fan_in = int(np.prod(s[1:])) if len(s) > 1 else 1
        sd = scale if scale is not None else (np.sqrt(2.0 / fan_in) if len(s) > 1 else 0.1)
        out[k] = rng.normal(0, sd, s)
    return out


def test_conv_forward_matches_direct_sum():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 5, 7, 3))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    y = cnn.conv_forward(x, w, b)
    assert y.shape == (2, 3, 4, 4)
    ref = np.zeros_like(y)
    for bb in range(2):
        for yo in range(3):
            for xo in range(4):
                for o in range(4):
                    s = b[o]
                    for c in range(3):
                        for ky in range(3):
                            for kx in range(3):
                                yy, xx = 2 * yo + ky - 1, 2 * xo + kx - 1
                                if 0 <= yy < 5 and 0 <= xx < 7:
                                    s += w[o, c, ky, kx] * x[bb, yy, xx, c]
                    ref[bb, yo, xo, o] = s
    assert np.abs(y - ref).max() < 1e-12


def _fd_check(shapes, S, c_in, B, coords_per_tensor=None, seed=1, weighted=False):
    rng = np.random.default_rng(seed)
    p = _rand_params(shapes, rng)
    x = rng.normal(size=(B, S, S, c_in))
    t = rng.normal(size=(B, shapes["fb2"][0]))
    w = rng.uniform(0.2, 3.0, B) if weighted else None
    loss, g, _ = cnn.loss_and_grads(p, x, t, weights=w)
    h = 1e-6
    worst = 0.0
    for k in cnn.PARAM_ORDER:
        flat = p[k].ravel()
        idx = range(flat.size) if coords_per_tensor is None else \
            rng.choice(flat.size, size=min(coords_per_tensor, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp = cnn.mse(cnn.forward(p, x)[0], t, w)[0]
            flat[i] = old - h
            lm = cnn.mse(cnn.forward(p, x)[0], t, w)[0]
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].ravel()[i]
            # relative error with an absolute floor for the central
            # difference's rounding noise (~eps / h = 1e-10)
            worst = max(worst, abs(fd - an) / (abs(fd) + abs(an) + 1e-4))
    return worst


def test_backward_matches_finite_differences_small_net():
    shapes = cnn.param_shapes(S=9, c_in=4, chans=(2, 3, 3), hidden=5, n_out=4)
    assert shapes["fw1"] == (5, 2 * 2 * 3)          # 9 -> 5 -> 3 -> 2
    assert _fd_check(shapes, S=9, c_in=4, B=3) < 1e-6


def test_weighted_loss_gradients_and_unit_weights():
    shapes = cnn.param_shapes(S=9, c_in=4, chans=(2, 3, 3), hidden=5, n_out=4)
    assert _fd_check(shapes, S=9, c_in=4, B=3, weighted=True) < 1e-6
    rng = np.random.default_rng(3)
    pred, t = rng.normal(size=(4, 6)), rng.normal(size=(4, 6))
    l1, g1 = cnn.mse(pred, t)
    l2, g2 = cnn.mse(pred, t, np.ones(4))
    assert l1 == l2 and np.array_equal(g1, g2)
    l3, _ = cnn.mse(pred, t, np.array([1.0, 0.0, 0.0, 0.0]))
    assert np.isclose(l3, np.sum((pred[0] - t[0]) ** 2) / pred.size)


def test_backward_matches_finite_differences_full_size_sampled():
    shapes = cnn.param_shapes()
    assert shapes["fw1"] == (2048, 1600)
    assert _fd_check(shapes, S=40, c_in=4, B=2, coords_per_tensor=6) < 1e-5


def test_adam_closed_form():
    w, g = np.array([1.0, -2.0, 0.5]), np.array([0.3, -4.0, 0.0])
    m = v = np.zeros(3)
    lr, eps = 0.01, 1e-8
    w1, m, v = cnn.adam_step(w, g, m, v, 1, lr, eps=eps)
    assert np.allclose(w1, w - lr * g / (np.abs(g) + eps), atol=1e-15)
    # With a constant gradient the bias-corrected moments stay g and g^2.
    w2, m, v = cnn.adam_step(w1, g, m, v, 2, lr, eps=eps)
    assert np.allclose(w2, w1 - lr * g / (np.abs(g) + eps), atol=1e-14)


def test_network_input_normalisation():
    rng = np.random.default_rng(2)
    S = 6
    ref = rng.uniform(0.5, 1.5, (4, S, S))
    valid = np.array([7, 8, 13, 14, 20, 27])
    x0 = cnn.network_input(ref[None] * 3.0, ref, valid)
    assert x0.shape == (1, S, S, 4) and np.abs(x0).max() < 1e-15
    p = rng.uniform(0.5, 1.5, (2, 4, S, S))
    x1 = cnn.network_input(p, ref, valid)
    x2 = cnn.network_input(p * 11.0, ref, valid)
    assert np.allclose(x1, x2, atol=1e-15)
    mask = np.zeros(S * S, bool); mask[valid] = True
    assert np.all(x1.reshape(2, S * S, 4)[:, ~mask] == 0)
    # Hand value: frame total flux mean over V is 4 (all ones), reference likewise.
    ones = np.ones((1, 4, S, S))
    p3 = ones.copy(); p3[0, 1, 1, 1] = 5.0           # j = 7 is valid: total 8 there
    x3 = cnn.network_input(p3, ones[0], valid)
    n = (4 * 6 + 4) / 6
    assert np.isclose(x3[0, 1, 1, 1], 5.0 / n - 0.25)
    assert np.isclose(x3[0, 1, 1, 0], 1.0 / n - 0.25)


def test_kl_coefficients_round_trip():
    A = pupil_amplitude(16)
    B = kl_modes(A, 0.25, 20.0, 12, cache=False)
    c = np.random.default_rng(3).normal(0, 50, (3, 12))
    opd = np.tensordot(c, B, axes=1)
    assert np.abs(cnn.kl_coefficients(opd, B, A) - c).max() < 1e-10


def test_adam_training_reduces_loss():
    shapes = cnn.param_shapes(S=9, c_in=4, chans=(3, 4, 4), hidden=16, n_out=3)
    rng = np.random.default_rng(4)
    p = _rand_params(shapes, rng, 0.2)
    x = rng.normal(size=(16, 9, 9, 4))
    t = rng.normal(size=(16, 3))
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    l0 = cnn.loss_and_grads(p, x, t)[0]
    for step in range(1, 101):
        _, g, _ = cnn.loss_and_grads(p, x, t)
        for k in p:
            p[k], m[k], v[k] = cnn.adam_step(p[k], g[k], m[k], v[k], step, 3e-3)
    assert cnn.loss_and_grads(p, x, t)[0] < 0.5 * l0


def test_bf16_round_values():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 0.0, 3.14159])
    r = cnn.bf16_round(v)
    # exact values on the bf16 grid stay; halfway cases go to even; relative error <= 2^-8
    assert r[0] == 1.0 and r[3] == -2.5 and r[4] == 0.0
    assert cnn.bf16_round(np.array([1.0 + 2 ** -7]))[0] == 1.0 + 2 ** -7
    assert cnn.bf16_round(np.array([1.0 + 2 ** -8]))[0] == 1.0                 # tie -> even (1.0)
    assert cnn.bf16_round(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6    # tie -> even
    assert np.all(np.abs(r - v) <= 2 ** -8 * np.abs(v))
