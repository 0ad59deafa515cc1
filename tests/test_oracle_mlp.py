"""Pins of the float64 network oracle: backpropagation against central finite
differences, closed forms of a network reduced to a linear map, and the
defining properties of the first Adam step."""
import numpy as np
import pytest

from oracle import mlp


def _data(seed, n=37):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, mlp.N_IN)), rng.normal(size=(n, mlp.N_OUT))


def test_parameter_count():
    assert mlp.N_PARAMS == 16 * 64 + 64 + 64 * 64 + 64 + 2 * 64 + 2 == 5378


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_central_differences(seed):
    x, t = _data(seed)
    th = mlp.init_params(seed)
    _, g = mlp.grad(th, x, t)
    rng = np.random.default_rng(seed + 10)
    idx = rng.choice(mlp.N_PARAMS, size=60, replace=False)
    h = 1e-6
    for k in idx:
        e = np.zeros_like(th)
        e[k] = h
        fd = (mlp.loss(th + e, x, t) - mlp.loss(th - e, x, t)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def test_linear_regime_closed_form():
    """With W1 = W2 = 0 the hidden layers are tanh(b) constants and the output
    is W3 tanh(b2) + b3: check forward and the output-layer gradient by hand."""
    p = mlp.unpack(mlp.init_params(3).copy())
    p["W1"][:] = 0
    p["W2"][:] = 0
    th = mlp.pack(p)
    x, t = _data(5, n=4)
    y, _ = mlp.forward(th, x)
    h2 = np.tanh(p["b2"])
    np.testing.assert_allclose(y, np.tile(p["W3"] @ h2 + p["b3"], (4, 1)), rtol=1e-14)
    _, g = mlp.grad(th, x, t)
    G = mlp.unpack(g)
    np.testing.assert_allclose(G["b3"], 2 * (y - t).sum(0) / 4, rtol=1e-13)
    np.testing.assert_allclose(G["W3"], np.outer(2 * (y - t).sum(0) / 4, h2), rtol=1e-13)
    assert not G["W1"].any() or np.allclose(G["W1"], 0.0)   # dh1/dW1 has x but W2 = 0 blocks it


def test_first_adam_step_moves_by_lr_sign():
    """After bias correction the first step is -lr g / (|g| + eps)."""
    rng = np.random.default_rng(0)
    th = rng.normal(size=100)
    g = rng.normal(size=100)
    new, m, v = mlp.adam_step(th, g, np.zeros(100), np.zeros(100), 1, 1e-2)
    np.testing.assert_allclose(new, th - 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_training_reduces_loss():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(256, mlp.N_IN))
    t = np.stack([np.sin(x[:, 0]) - 0.5 * x[:, 1], 0.3 * x[:, 2] * x[:, 3]], axis=1)
    th = mlp.init_params(0)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    l0 = mlp.loss(th, x, t)
    for k in range(1, 301):
        _, g = mlp.grad(th, x, t)
        th, m, v = mlp.adam_step(th, g, m, v, k, 3e-3)
    assert mlp.loss(th, x, t) < 0.2 * l0
