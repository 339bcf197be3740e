"""Pins of the FP64 estimator reference: closed forms and finite differences."""
import numpy as np
import pytest

from oracle import mlp as M


def _rand_params(seed):
    rng = np.random.default_rng(seed)
    p = {}
    for k in M.ORDER:
        fan = M.SHAPES[k][-1] if len(M.SHAPES[k]) == 2 else 64
        p[k] = rng.standard_normal(M.SHAPES[k]) / np.sqrt(fan)
    return p


def test_closed_form_identity_network():
    """Hidden layers pass the positive part of the inputs through; the output
    sums them with weights w3, so y = sum_j w3_j relu(x_j) + b3 by hand."""
    p = {k: np.zeros(s) for k, s in M.SHAPES.items()}
    p["W1"][:18, :18] = np.eye(18)
    p["W2"][:18, :18] = np.eye(18)
    p["w3"][:18] = np.arange(1, 19, dtype=np.float64)
    p["b3"][0] = 0.5
    X = np.array([np.linspace(-1, 1, 18), np.full(18, 2.0)])
    y, _ = M.forward(p, X)
    want0 = sum((j + 1) * max(v, 0.0) for j, v in enumerate(X[0])) + 0.5
    want1 = 2.0 * sum(range(1, 19)) + 0.5
    assert y[0] == pytest.approx(want0, rel=1e-15)
    assert y[1] == pytest.approx(want1, rel=1e-15)
    # loss against z: mean of squared residuals
    assert M.loss(p, X, [want0 - 1.0, want1 + 3.0]) == pytest.approx((1.0 + 9.0) / 2)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = _rand_params(2)
    X = rng.standard_normal((7, 18))
    z = rng.uniform(0, 10, 7)
    _, g = M.loss_and_grad(p, X, z)
    fd = M.finite_difference(p, X, z, h=1e-6)
    an = M.flatten(g)
    # relu kinks are measure-zero for random inputs; central differences are O(h^2)
    rel = np.linalg.norm(an - fd) / np.linalg.norm(fd)
    assert rel < 1e-6
    assert M.n_params() == 64 * 18 + 64 + 64 * 64 + 64 + 64 + 1


def test_gradient_bias_only_closed_form():
    """With all weights zero the network is the constant b3; dL/db3 = 2 mean(b3 - z)."""
    p = {k: np.zeros(s) for k, s in M.SHAPES.items()}
    p["b3"][0] = 4.0
    z = np.array([1.0, 2.0, 6.0])
    L, g = M.loss_and_grad(p, np.ones((3, 18)), z)
    assert L == pytest.approx(((3.0) ** 2 + 2.0 ** 2 + 2.0 ** 2) / 3)
    assert g["b3"][0] == pytest.approx(2.0 * np.mean(4.0 - z))
    for k in ("W1", "b1", "W2", "b2", "w3"):
        assert not np.any(g[k])


def test_adam_first_step_is_signed_lr():
    """At t = 1 the bias-corrected moments are g and g^2, so the step is
    lr * g / (|g| + eps)."""
    p = _rand_params(3)
    g = _rand_params(4)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(x) for k, x in p.items()}
    before = {k: x.copy() for k, x in p.items()}
    M.adam_step(p, g, m, v, 1, lr=0.01)
    for k in M.ORDER:
        want = before[k] - 0.01 * g[k] / (np.abs(g[k]) + 1e-8)
        assert np.allclose(p[k], want, rtol=1e-12, atol=1e-15)


def test_training_reduces_loss():
    rng = np.random.default_rng(6)
    X = rng.standard_normal((256, 18))
    z = np.tanh(X[:, 0]) * 3 + X[:, 1] ** 2
    p = _rand_params(7)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(x) for k, x in p.items()}
    L0 = M.loss(p, X, z)
    for t in range(1, 201):
        _, g = M.loss_and_grad(p, X, z)
        M.adam_step(p, g, m, v, t, lr=3e-3)
    assert M.loss(p, X, z) < 0.2 * L0
