"""Pins for the FP64 warm-start references in oracle/mlp.py."""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import mlp


def rand_params(seed, scale=0.3):
    return np.random.default_rng(seed).normal(0, scale, mlp.NPARAMS)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_backward_matches_central_differences(seed):
    rng = np.random.default_rng(seed)
    p = rand_params(seed)
    X = rng.normal(0, 1, (48, mlp.F))
    t = rng.normal(0, 1, 48)
    loss, g = mlp.loss_and_grad(p, X, t)
    h = 1e-6
    for i in rng.choice(mlp.NPARAMS, 60, replace=False):
        e = np.zeros(mlp.NPARAMS)
        e[i] = h
        fd = (mlp.loss_and_grad(p + e, X, t)[0] - mlp.loss_and_grad(p - e, X, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), i


def test_forward_special_cases():
    X = np.random.default_rng(4).normal(0, 1, (10, mlp.F))
    w = mlp.unpack(rand_params(5))
    w["W2"][:] = 0.0  # second layer sees only its bias
    p = mlp.pack(w)
    y, _ = mlp.forward(p, X)
    np.testing.assert_allclose(y, w["w3"] @ np.maximum(w["b2"], 0) + w["b3"][0])
    # all-negative pre-activations: output is b3 and only b3 gets a gradient
    w = mlp.unpack(rand_params(6))
    w["W1"][:] = 0.0
    w["b1"][:] = -1.0
    w["b2"][:] = -1.0  # h1 = 0 makes a2 = b2
    p = mlp.pack(w)
    y, _ = mlp.forward(p, X)
    np.testing.assert_allclose(y, w["b3"][0])
    _, g = mlp.loss_and_grad(p, X, np.zeros(10))
    gd = mlp.unpack(g)
    assert np.all(gd["W1"] == 0) and np.all(gd["W2"] == 0) and gd["b3"][0] != 0


def test_adam_first_step_moves_by_lr_sign():
    """With zero moments and bias correction, step 1 is lr * g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p, m, v = mlp.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    np.testing.assert_allclose(p[:3], -0.01 * np.sign(g[:3]), rtol=1e-4)
    assert p[3] == 0.0


def test_adam_constant_gradient_moves_by_lr_every_step():
    """With bias correction, a constant gradient g gives m_t / (1 - b1^t) = g
    and v_t / (1 - b2^t) = g^2 at every step t, so each step moves by
    lr * sign(g) (eps = 0)."""
    g = np.array([2.0, -0.25])
    p, m, v = np.zeros(2), np.zeros(2), np.zeros(2)
    for t in range(1, 6):
        p, m, v = mlp.adam_step(p, g, m, v, t, 0.1, eps=0.0)
        np.testing.assert_allclose(p, -0.1 * t * np.sign(g), rtol=1e-13)


def test_adam_second_step_by_hand():
    """Gradient +1 then -1, lr 0.1, b1 0.9, b2 0.999, eps 0, worked by hand:
    step 1: m = 0.1, v = 0.001, corrected 1 and 1, p = -0.1;
    step 2: m = 0.09 - 0.1 = -0.01, corrected -0.01 / 0.19; v = 0.000999 +
    0.001 = 0.001999, corrected 0.001999 / 0.001999 = 1; p = -0.1 + 0.1 *
    0.01 / 0.19 = -0.0947368421052631...  With b1 and b2 swapped the second
    step would give -0.1 + 0.1 * 1e-6 / 0.001999 instead."""
    p, m, v = mlp.adam_step(np.zeros(1), np.ones(1), np.zeros(1), np.zeros(1), 1, 0.1, eps=0.0)
    np.testing.assert_allclose(p, [-0.1], rtol=1e-15)
    p, m, v = mlp.adam_step(p, -np.ones(1), m, v, 2, 0.1, eps=0.0)
    np.testing.assert_allclose(m, [-0.01], rtol=1e-12)
    np.testing.assert_allclose(v, [0.001999], rtol=1e-12)
    np.testing.assert_allclose(p, [-0.1 + 0.001 / 0.19], rtol=1e-13)
    np.testing.assert_allclose(p, [-0.09473684210526316], rtol=1e-13)


def test_features_from_definitions():
    """Feature 3 is log(n PR_1) of the first PageRank iterate from 1/n."""
    r, c = graphgen.rmat(10, 8, seed=2, relabel="random")
    n = len(r) - 1
    X = mlp.features(r, c)
    pr1 = oracle.pagerank(r, c, iters=1).x
    np.testing.assert_allclose(X[:, 3], np.log(n * pr1), rtol=1e-12, atol=1e-12)
    assert X[:, 2].sum() == (np.diff(r) == 0).sum()
    np.testing.assert_allclose(np.expm1(X[:, 0]).sum(), len(c))
    assert np.all(X[:, 4:] == 0)
