"""Pins of the FP64 predictor-network oracle against closed forms and finite
differences (independent of its own chain-rule code)."""
import numpy as np
import pytest

import oracle.mlp as OM


def test_parameter_count_and_layout():
    assert OM.param_count() == 128 * 258 + 128 + 128 * 128 + 128 + 2 * 128 + 2 == 49922
    theta = np.arange(OM.param_count(), dtype=float)
    W1, b1, W2, b2, W3, b3 = OM.unflatten(theta)
    assert W1[1, 0] == 258 and b1[0] == 128 * 258 and W3.shape == (2, 128) and b3[-1] == 49921


def test_forward_closed_form_abs_sum():
    # h1 = [relu(x_i), relu(-x_i)] for i < 64; h2[0] = sum |x_i|; y = (h2[0], 3)
    W1 = np.zeros((128, 258))
    W1[np.arange(64), np.arange(64)] = 1.0
    W1[64 + np.arange(64), np.arange(64)] = -1.0
    W2 = np.zeros((128, 128))
    W2[0, :] = 1.0
    W3 = np.zeros((2, 128))
    W3[0, 0] = 1.0
    b3 = np.array([0.0, 3.0])
    theta = np.concatenate([W1.ravel(), np.zeros(128), W2.ravel(), np.zeros(128), W3.ravel(), b3])
    X = np.random.default_rng(1).standard_normal((5, 258))
    y, _ = OM.forward(theta, X)
    assert np.allclose(y[:, 0], np.abs(X[:, :64]).sum(axis=1), rtol=0, atol=1e-13)
    assert np.all(y[:, 1] == 3.0)


def test_loss_zero_at_own_output_and_quadratic():
    theta = OM.init_params(3)
    X = np.random.default_rng(2).uniform(-1, 1, (9, 258))
    y, _ = OM.forward(theta, X)
    assert OM.loss(theta, X, y) == 0.0
    assert abs(OM.loss(theta, X, y + 2.0) - 0.5 * 2 * 4.0) < 1e-12     # two outputs, shift 2, mean over batch


@pytest.mark.parametrize("B", [1, 6])
def test_gradient_matches_central_differences(B):
    rng = np.random.default_rng(B)
    theta = OM.init_params(10 + B)
    theta[33024:33024 + 128] = rng.uniform(0.05, 0.2, 128)   # b1 > 0 keeps most units active
    X = rng.uniform(-1, 1, (B, 258))
    T = rng.standard_normal((B, 2))
    _, g = OM.gradient(theta, X, T)
    h = 1e-6
    # every bias, and random weights of each layer
    idx = list(range(33024, 33152)) + list(range(49536, 49664)) + [49920, 49921]
    for lo, hi in [(0, 33024), (33152, 49536), (49664, 49920)]:
        idx += list(rng.integers(lo, hi, 60))
    for k in idx:
        e = np.zeros_like(theta)
        e[k] = h
        fd = (OM.loss(theta + e, X, T) - OM.loss(theta - e, X, T)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), k


def test_adam_closed_forms():
    # first step: m^ = g, v^ = g^2 -> step lr g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    th = np.zeros(4)
    t1, m, v = OM.adam(th, g, np.zeros(4), np.zeros(4), 1, lr=0.1, eps=1e-8)
    assert np.allclose(t1, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=0)
    # a constant gradient keeps the bias-corrected moments at g and g^2 on every step
    t, m, v = th, np.zeros(4), np.zeros(4)
    for step in range(1, 6):
        t, m, v = OM.adam(t, g, m, v, step, lr=0.1, eps=0.0 + 1e-300)
    nz = g != 0
    assert np.allclose(t[nz], -0.5 * np.sign(g[nz]), rtol=1e-12)
    assert t[~nz][0] == 0.0


def test_training_fits_linear_target():
    rng = np.random.default_rng(0)
    X = rng.uniform(-1, 1, (64, 258))
    T = np.stack([X[:, 0] - 0.5 * X[:, 1], X[:, 2]], axis=1)
    theta = OM.init_params(4)
    m, v = np.zeros_like(theta), np.zeros_like(theta)
    l0 = OM.loss(theta, X, T)
    for step in range(1, 301):
        _, g = OM.gradient(theta, X, T)
        theta, m, v = OM.adam(theta, g, m, v, step, lr=1e-3)
    assert OM.loss(theta, X, T) < 0.05 * l0
