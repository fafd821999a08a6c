"""Pins for the oracle's cost-model MLP (forward, loss gradient, Adam) and its
error statistics.

MLP gradient: central finite differences.  Forward: a numpy restatement on a
tiny network.  Adam: the step-1 closed form (with bias correction the first
update is -lr * g / (|g| + eps)), a two-step hand computation, and convergence
on a quadratic.  Error statistics: hand-computed small cases.
"""
import numpy as np
import pytest

D0, H1, H2 = 6, 8, 5


def _params(orc, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(orc.mlp_param_count(D0, H1, H2)) * 0.5


def test_param_count(orc):
    assert orc.mlp_param_count(D0, H1, H2) == D0 * H1 + H1 + H1 * H2 + H2 + H2 + 1


def test_forward_matches_numpy(orc):
    p = _params(orc, 0)
    X = np.random.default_rng(1).standard_normal((7, D0))
    o = 0
    W1 = p[o:o + D0 * H1].reshape(D0, H1); o += D0 * H1
    b1 = p[o:o + H1]; o += H1
    W2 = p[o:o + H1 * H2].reshape(H1, H2); o += H1 * H2
    b2 = p[o:o + H2]; o += H2
    W3 = p[o:o + H2]; o += H2
    b3 = p[o]
    h = np.maximum(X @ W1 + b1, 0)
    h = np.maximum(h @ W2 + b2, 0)
    want = h @ W3 + b3
    np.testing.assert_allclose(orc.mlp_forward(p, X, H1, H2), want, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_vs_central_differences(orc, seed):
    p = _params(orc, seed)
    rng = np.random.default_rng(seed + 10)
    X = rng.standard_normal((9, D0))
    t = rng.standard_normal(9)
    loss, g = orc.mlp_loss_grad(p, X, t, H1, H2)
    y = orc.mlp_forward(p, X, H1, H2)
    assert abs(loss - np.mean((y - t) ** 2)) < 1e-12
    h = 1e-6
    num = np.empty_like(p)
    for i in range(p.size):
        pp = p.copy(); pp[i] += h
        pm = p.copy(); pm[i] -= h
        num[i] = (orc.mlp_loss_grad(pp, X, t, H1, H2)[0] - orc.mlp_loss_grad(pm, X, t, H1, H2)[0]) / (2 * h)
    rel = np.linalg.norm(g - num) / np.linalg.norm(num)
    assert rel < 1e-6


def test_adam_first_step_closed_form(orc):
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 0.01, 1e-8
    orc.adam_step(p, g, m, v, lr, 0.9, 0.999, eps, 1)
    np.testing.assert_allclose(p, -lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)


def test_adam_two_steps_by_hand(orc):
    g1, g2 = 0.5, -0.25
    b1, b2, lr, eps = 0.9, 0.999, 0.1, 1e-8
    p = np.zeros(1); m = np.zeros(1); v = np.zeros(1)
    orc.adam_step(p, np.array([g1]), m, v, lr, b1, b2, eps, 1)
    orc.adam_step(p, np.array([g2]), m, v, lr, b1, b2, eps, 2)
    m1 = (1 - b1) * g1; v1 = (1 - b2) * g1 ** 2
    p1 = -lr * (m1 / (1 - b1)) / (np.sqrt(v1 / (1 - b2)) + eps)
    m2 = b1 * m1 + (1 - b1) * g2; v2 = b2 * v1 + (1 - b2) * g2 ** 2
    p2 = p1 - lr * (m2 / (1 - b1 ** 2)) / (np.sqrt(v2 / (1 - b2 ** 2)) + eps)
    assert abs(p[0] - p2) < 1e-14


def test_training_reduces_loss(orc):
    rng = np.random.default_rng(3)
    X = rng.standard_normal((64, D0))
    t = np.sin(X[:, 0]) + 0.5 * X[:, 1] ** 2
    p = _params(orc, 4) * 0.5
    m = np.zeros_like(p); v = np.zeros_like(p)
    l0, _ = orc.mlp_loss_grad(p, X, t, H1, H2)
    for step in range(1, 301):
        _, g = orc.mlp_loss_grad(p, X, t, H1, H2)
        orc.adam_step(p, g, m, v, 0.01, 0.9, 0.999, 1e-8, step)
    l1, _ = orc.mlp_loss_grad(p, X, t, H1, H2)
    assert l1 < 0.3 * l0


def test_err_stats_by_hand(orc):
    c = np.array([1.0, 2.0, 4.0])
    r = np.array([1.0, 3.0, 2.0])
    bound = np.array([1.0, 0.5, 0.0])
    s = orc.err_stats(c, r, bound)
    assert list(s) == [0 + 1 + 4, 1 + 9 + 4, 2.0, 2.0]
    assert orc.normwise_rel_err(c, r) == pytest.approx(np.sqrt(5 / 14), rel=1e-15)
    assert orc.err_stats(c, r)[3] == 0.0
