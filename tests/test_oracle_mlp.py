"""Pins of the FP64 cost-model reference: central finite differences for the
hand-written backprop, closed forms for the forward pass and for Adam."""
import numpy as np
import pytest

from oracle import mlp_ref as M


def test_parameter_count():
    assert M.N_PARAMS == 12 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 5057


def test_forward_closed_forms():
    theta = np.zeros(M.N_PARAMS)
    parts = M.unpack(theta)
    parts["b3"][:] = 3.25
    X = np.random.default_rng(0).normal(size=(5, 12))
    yhat, _ = M.forward(M.pack(parts), X, np.zeros(12), np.ones(12))
    assert np.allclose(yhat, 3.25)           # no hidden activity: output is the bias
    # one path: unit 0 of each layer passes x0 through, output = 2 * relu(relu(x0 - 1) + 0.5)
    parts = M.unpack(np.zeros(M.N_PARAMS))
    parts["W1"][0, 0] = 1.0
    parts["b1"][0] = -1.0
    parts["W2"][0, 0] = 1.0
    parts["b2"][0] = 0.5
    parts["W3"][0] = 2.0
    x = np.zeros((3, 12))
    x[:, 0] = [0.0, 1.5, 4.0]
    yhat, _ = M.forward(M.pack(parts), x, np.zeros(12), np.ones(12))
    assert np.allclose(yhat, [1.0, 2.0, 7.0])
    # normalisation is applied before the first layer
    mu, sd = np.full(12, 2.0), np.full(12, 4.0)
    x2 = x * 4.0 + 2.0
    assert np.allclose(M.forward(M.pack(parts), x2, mu, sd)[0], yhat)


@pytest.mark.parametrize("seed", range(3))
def test_backprop_matches_central_differences(seed):
    rng = np.random.default_rng(seed)
    theta = M.init(seed)
    X = rng.normal(size=(17, 12)) * 3 + 1
    y = rng.normal(size=17)
    mu, sd = X.mean(0), X.std(0) + 0.5
    g, _ = M.grad(theta, X, y, mu, sd)
    idx = rng.choice(M.N_PARAMS, size=60, replace=False)
    idx = np.concatenate([idx, [0, 767, 768, 831, 832, 4927, 4928, 4991, 4992, 5055, 5056]])
    eps = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (M.loss(tp, X, y, mu, sd) - M.loss(tm, X, y, mu, sd)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_adam_first_step_closed_form():
    # with zero moments the first bias-corrected step is lr * g / (|g| + eps)
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    t1, m, v = M.adam_step(theta, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(t1, theta - 0.01 * g / (np.abs(g) + 1e-8))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_training_reduces_loss():
    rng = np.random.default_rng(4)
    X = rng.uniform(0, 10, size=(256, 12))
    y = 0.3 * X[:, 0] - 0.2 * X[:, 3] + np.sin(X[:, 5])
    mu, sd = X.mean(0), X.std(0)
    theta = M.init(1)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = M.loss(theta, X, y, mu, sd)
    for t in range(1, 301):
        g, _ = M.grad(theta, X, y, mu, sd)
        theta, m, v = M.adam_step(theta, g, m, v, t, lr=3e-3)
    assert M.loss(theta, X, y, mu, sd) < 0.1 * l0
