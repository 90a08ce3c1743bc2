"""Pins of the FP64 MLP oracle: back-propagated gradients equal central finite
differences of the loss; SiLU derivative; features of special states;
Adam's first step has magnitude lr per weight (sign of the gradient)."""
import numpy as np
import pytest

from oracle import mlp as M


def _params(seed):
    rng = np.random.default_rng(seed)
    p = np.zeros(M.NP)
    p[:M.NW] = rng.uniform(-0.4, 0.4, M.NW)
    p[M.O_MU:M.O_MU + 5] = rng.uniform(-1, 1, 5)
    p[M.O_SD:M.O_SD + 5] = rng.uniform(0.5, 2, 5)
    p[M.O_YMU] = 0.3
    p[M.O_YSD] = 1.7
    return p


def test_silu_derivative_matches_finite_difference():
    a = np.linspace(-8, 8, 101)
    h = 1e-6
    fd = (M.silu(a + h) - M.silu(a - h)) / (2 * h)
    assert np.abs(fd - M.dsilu(a)).max() < 1e-8


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    p = _params(2)
    x = rng.normal(size=(5, 37))
    t = rng.normal(size=37)
    L, g = M.loss_and_grad(p, x, t)
    assert abs(L - M.loss(p, x, t)) < 1e-15 * max(1.0, L)
    idx = np.concatenate([rng.choice(M.NW, 200, replace=False), [M.O_B3, M.O_B1, M.O_B2, M.O_W3]])
    for k in idx:
        h = 1e-6 * max(1.0, abs(p[k]))
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (M.loss(pp, x, t) - M.loss(pm, x, t)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(np.abs(g).max(), 1e-12) + 1e-9, (k, fd, g[k])


def test_forward_of_zero_network_is_bias():
    p = np.zeros(M.NP)
    p[M.O_SD:M.O_SD + 5] = 1.0
    p[M.O_YSD] = 2.0
    p[M.O_YMU] = 0.5
    p[M.O_B3] = 0.25
    y = M.predict(p, np.ones((5, 3)))
    assert np.allclose(y, 0.25 * 2.0 + 0.5)


def test_features_of_special_states(ora):
    g = 4.0 / 3.0
    # hydro at rest: |S| = 0, B = 0 -> f(0) = (g-1) tau, so the last feature is ln((g-1) tau/D)
    U = np.array([[2.0], [0.0], [0.0], [0.0], [3.0]])
    f = M.features(1, g, U)
    assert np.allclose(f[:, 0], [np.log(1.5), 0.0, 0.0, 0.0, np.log((g - 1) * 1.5)], rtol=0, atol=1e-15)
    # MHD with S parallel to B: cosine feature is 1
    U = np.array([[1.0], [0.3], [0.0], [0.0], [2.0], [0.7], [0.0], [0.0], [0.0]])
    f = M.features(2, g, U)
    assert abs(f[3, 0] - 1.0) < 1e-12
    assert abs(f[2, 0] - np.log1p(0.49)) < 1e-15
    # a cold state (p -> 0) has f(0) -> 0: the last feature tracks ln(p/D)
    prim = np.array([[1.0], [0.3], [0.1], [0.0], [1e-8]])
    U = ora.prim2cons(1, g, prim)
    assert abs(M.features(1, g, U)[4, 0] - np.log(1e-8 / U[0, 0])) < 0.05


def test_adam_first_step_is_lr_times_sign():
    rng = np.random.default_rng(4)
    p = _params(5)
    g = rng.normal(size=M.NW)
    p1, m, v = M.adam_step(p, g, np.zeros(M.NW), np.zeros(M.NW), 1, 1e-3)
    # with bias correction the first step is lr g / (|g| + eps): lr sign(g) up to eps
    assert np.allclose((p - p1)[:M.NW], 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)
    assert np.array_equal(p1[M.NW:], p[M.NW:])
