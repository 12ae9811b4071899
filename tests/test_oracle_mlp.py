"""Pins of the oracle's selector network: closed-form derivatives and central
finite differences of the FP64 loss."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_gelu_closed_values():
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert mlp.gelu_grad(np.array([0.0]))[0] == 0.5
    x = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.allclose(fd, mlp.gelu_grad(x), rtol=1e-8, atol=1e-9)
    # large |x|: GELU -> relu
    assert abs(mlp.gelu(np.array([10.0]))[0] - 10.0) < 1e-12


def test_softmax_ce_gradient_closed_form():
    params = mlp.init_params(0)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((7, 8))
    y = rng.integers(0, 4, 7)
    W3 = params[4]
    logits, (X_, a1, h1, a2, h2) = mlp.forward(params, X)
    P = mlp.softmax(logits)
    onehot = np.eye(4)[y]
    _, grads = mlp.loss_and_grads(params, X, y)
    # dL/db3 = mean(p - onehot), dL/dW3 = (p - onehot)^T h2 / B
    assert np.allclose(grads[5], (P - onehot).mean(axis=0), atol=1e-15)
    assert np.allclose(grads[4], (P - onehot).T @ h2 / 7, atol=1e-14)


@pytest.mark.parametrize("seed", [0, 1])
def test_finite_differences_all_parameters(seed):
    params = mlp.init_params(seed)
    rng = np.random.default_rng(10 + seed)
    X = rng.standard_normal((5, 8))
    y = rng.integers(0, 4, 5)
    loss, grads = mlp.loss_and_grads(params, X, y)
    h = 1e-6
    for pi, (p, g) in enumerate(zip(params, grads)):
        flat = p.ravel()
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp, _ = mlp.loss_and_grads(params, X, y)
            flat[i] = old - h
            lm, _ = mlp.loss_and_grads(params, X, y)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            gi = g.ravel()[i]
            assert abs(fd - gi) <= 1e-6 * max(1e-3, abs(gi)) + 1e-9, (pi, i, fd, gi)


def test_predict_ties_to_lower_rung():
    params = mlp.init_params(0)
    for i in range(0, 6, 2):
        params[i][:] = 0.0
    params[5][:] = np.array([0.0, 1.0, 1.0, 0.5])
    assert list(mlp.predict(params, np.zeros((2, 8)))) == [1, 1]


def test_adam_first_step():
    p = [np.array([1.0, -2.0])]
    g = [np.array([0.5, -4.0])]
    st = {}
    mlp.adam_step(p, g, st, lr=0.1)
    # first step: m_hat = g, v_hat = g^2 -> p -= lr * g / (|g| + eps)
    assert np.allclose(p[0], [1.0 - 0.1 * 0.5 / (0.5 + 1e-8), -2.0 + 0.1 * 4 / (4 + 1e-8)])


def test_he_init_scale():
    params = mlp.init_params(3, sizes=(8, 4096, 2))
    assert abs(params[0].std() - math.sqrt(2 / 8)) < 0.02


def test_adam_constant_gradient_steps_are_lr_sign():
    # with a constant gradient the bias-corrected moments are exactly g and g^2
    # at every step, so each step moves by lr * g / (|g| + eps); a wrong bias
    # correction (or none) breaks this from the second step on
    p = [np.array([0.0, 0.0, 0.0])]
    g = [np.array([0.3, -2.0, 1e-3])]
    st = {}
    for t in range(1, 6):
        mlp.adam_step(p, g, st, lr=0.01)
        step = 0.01 * g[0] / (np.abs(g[0]) + 1e-8)
        assert np.allclose(p[0], -t * step, rtol=1e-12, atol=1e-15)
    assert st["t"] == 5


def test_adam_moments_follow_exponential_averages():
    # alternating gradients: m_t and v_t are the closed-form geometric sums
    p = [np.array([0.0])]
    st = {}
    gs = [1.0, -1.0, 1.0, -1.0]
    for g in gs:
        mlp.adam_step(p, [np.array([g])], st, lr=0.0)
    m = sum((1 - 0.9) * 0.9 ** (len(gs) - 1 - i) * gs[i] for i in range(len(gs)))
    v = sum((1 - 0.999) * 0.999 ** (len(gs) - 1 - i) * gs[i] ** 2 for i in range(len(gs)))
    assert abs(st["m"][0][0] - m) < 1e-15 and abs(st["v"][0][0] - v) < 1e-15
