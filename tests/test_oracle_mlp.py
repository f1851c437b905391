"""Pins of the FP64 learned-selector oracle (oracle/mlp_ref.py) against what mathematics
fixes: central finite differences of the loss, textbook values of the normal CDF, an
independent form of the binary cross-entropy, the closed form of Adam's first step and
of the geometric mean energy, and learning a separable toy problem."""
import math

import numpy as np
import pytest

from oracle import mlp_ref as M
from synthvideo import mlp_init


def test_parameter_count():
    assert M.NPARAM == 4673
    assert len(mlp_init(0)) == M.NPARAM


def test_gelu_textbook_values_and_symmetry():
    # GELU(x) = x Phi(x); Phi(1) = 0.8413447460685429, Phi(2) = 0.9772498680518208
    assert M.gelu(np.array(0.0)) == 0.0
    assert abs(M.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15
    assert abs(M.gelu(np.array(2.0)) - 2 * 0.9772498680518208) < 1e-15
    x = np.linspace(-6, 6, 101)
    np.testing.assert_allclose(M.gelu(-x), M.gelu(x) - x, atol=1e-14)
    # derivative against central differences
    h = 1e-6
    np.testing.assert_allclose(M.gelu_grad(x), (M.gelu(x + h) - M.gelu(x - h)) / (2 * h), atol=1e-8)


def test_bce_with_logits_matches_naive_form_and_is_stable():
    rng = np.random.default_rng(0)
    z = rng.normal(scale=4, size=200)
    y = (rng.random(200) < 0.5).astype(float)
    s = 1 / (1 + np.exp(-z))
    naive = -(y * np.log(s) + (1 - y) * np.log(1 - s))
    np.testing.assert_allclose(M.bce_with_logits(z, y), naive, rtol=1e-12)
    assert M.bce_with_logits(800.0, 1.0) == 0.0
    assert M.bce_with_logits(-800.0, 0.0) == 0.0
    assert M.bce_with_logits(800.0, 0.0) == 800.0


@pytest.mark.parametrize("seed", [1, 2])
def test_gradient_matches_finite_differences(seed):
    rng = np.random.default_rng(seed)
    theta = mlp_init(seed)
    X = rng.normal(size=(24, 6))
    y = (rng.random(24) < 0.4).astype(float)
    _, g = M.loss_and_grad(theta, X, y)
    # every block: W1, b1, W2, b2, w3, b3
    blocks = [(0, 384), (384, 448), (448, 4544), (4544, 4608), (4608, 4672), (4672, 4673)]
    idx = np.concatenate([rng.choice(np.arange(a, b), size=min(12, b - a), replace=False) for a, b in blocks])
    gn = M.numerical_grad(theta, X, y, h=1e-6, idx=idx)
    np.testing.assert_allclose(g[idx], gn, rtol=1e-5, atol=1e-9)


def test_adam_first_step_closed_form():
    """After bias correction the first moments are g and g^2: the step is
    -lr g / (|g| + eps), i.e. lr times the sign of g up to eps."""
    rng = np.random.default_rng(3)
    g = rng.normal(size=50)
    opt = M.Adam(50, lr=1e-3)
    th = opt.step(np.zeros(50), g)
    np.testing.assert_allclose(th, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-13)
    np.testing.assert_allclose(th, -1e-3 * np.sign(g), rtol=1e-5)


def test_features_closed_forms():
    m, k = 40, 4
    lam = np.array([1.0, 0.9 * np.exp(0.3j), 0.9 * np.exp(-0.3j), 1.02])
    b = np.array([2.0, 0.5 + 0.5j, 0.5 - 0.5j, 1e-3])
    phin = np.array([1.5, 2.0, 2.0, 0.7])
    x1 = 9.0
    F = M.features(lam, b, phin, x1, m)
    np.testing.assert_allclose(F[:, 0], np.abs(lam))
    np.testing.assert_allclose(F[:, 1], [0.0, 0.3, 0.3, 0.0], atol=1e-15)
    # |b_j| ||phi_j|| / ||x_1|| with ||x_1|| = 3: 2 * 1.5 / 3 = 1, (1/sqrt 2) * 2 / 3 = sqrt(2) / 3
    # and 1e-3 * 0.7 / 3
    np.testing.assert_allclose(F[:, 2], [0.0, np.log(np.sqrt(2.0) / 3.0), np.log(np.sqrt(2.0) / 3.0),
                                         np.log(7e-4 / 3.0)], atol=1e-15)
    np.testing.assert_allclose(F[:, 3], [0.75, 1.0, 1.0, 0.35])
    np.testing.assert_allclose(F[:, 5], np.arange(k) / k)
    # invariances: the scale of C moves b and phi in opposite directions; a larger frame
    # scales phi and x_1 together
    np.testing.assert_allclose(M.features(lam, 7.0 * b, phin / 7.0, x1, m), F, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(M.features(lam, b, 5.0 * phin, 25.0 * x1, m), F, rtol=1e-13, atol=1e-15)
    # |lambda| = 1: no decay; otherwise the geometric mean (1 - a^2m) / (m (1 - a^2))
    assert abs(F[0, 4] - 4.0 * 1.5 ** 2 / x1) < 1e-14
    a = 0.9
    geo = (1 - a ** (2 * m)) / (m * (1 - a * a))
    assert abs(F[1, 4] - 0.5 * 4.0 * geo / x1) < 1e-14
    a = 1.02
    geo = (a ** (2 * m) - 1) / (m * (a * a - 1))
    assert abs(F[3, 4] - 1e-6 * 0.49 * geo / x1) < 1e-18


def test_training_learns_a_separable_rule():
    rng = np.random.default_rng(5)
    X = rng.normal(size=(512, 6))
    y = (X[:, 0] - 0.5 * X[:, 2] > 0).astype(float)
    theta0 = mlp_init(5)
    batches = [rng.permutation(512)[:64] for _ in range(300)]
    theta = M.train(theta0, X, y, batches, lr=3e-3)
    assert M.loss(theta, X, y) < 0.25 * M.loss(theta0, X, y)
    pr, _, _ = M.predict(theta, X)
    assert ((pr >= 0.5) == (y > 0.5)).mean() > 0.95
