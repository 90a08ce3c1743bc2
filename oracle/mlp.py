"""FP64 reference of the pressure-guess network (test infrastructure only).

A 5 -> 64 -> 64 -> 1 multilayer perceptron with SiLU activations
s(a) = a sigma(a), sigma the logistic function, trained on the mean squared
error; textbook back-propagation and the Adam update (Kingma & Ba, with bias
correction).  The parameter layout is W1[64][5] b1[64] W2[64][64] b2[64]
W3[64] b3 (4609 weights) followed by mu[5] sd[5] ymu ysd (normalisation).

Inputs are five invariants of a conserved state (D, S_i, tau, B^i):
  [ln(tau/D), ln(1 + |S|/D), ln(1 + B^2/D), S.B / (|S||B| + tiny), ln(f(0)/D)]
with f the recovery's pressure function, and the target is ln(p/D).  Parity is pinned by central finite differences
of the loss (tests/test_oracle_mlp.py).
"""
from __future__ import annotations

import numpy as np

H, IN = 64, 5
O_W1, O_B1 = 0, 320
O_W2, O_B2 = 384, 4480
O_W3, O_B3 = 4544, 4608
NW = 4609
O_MU, O_SD, O_YMU, O_YSD = 4609, 4614, 4619, 4620
NP = 4621


def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    return (p[O_W1:O_B1].reshape(H, IN), p[O_B1:O_W2], p[O_W2:O_B2].reshape(H, H), p[O_B2:O_W3],
            p[O_W3:O_B3], p[O_B3])


def features(system, gamma, U):
    """Raw features [5][n] of conserved states U[nv][n] (B = 0 for hydro):
    [ln(tau/D), ln(1 + |S|/D), ln(1 + B^2/D), S.B/(|S||B| + tiny),
     ln(f(0)/D)], f the recovery's pressure function (the oracle's own), whose
    value at zero pressure, (gamma-1) rho eps(0), measures the thermal energy
    left after the kinetic and magnetic parts; ln of a floor 1e-300 where
    f(0) <= 0 or is undefined."""
    import oracle
    U = np.asarray(U, dtype=np.float64)
    D, tau = U[0], U[4]
    S2 = U[1] ** 2 + U[2] ** 2 + U[3] ** 2
    if system == 2:
        BB = U[5] ** 2 + U[6] ** 2 + U[7] ** 2
        SB = U[1] * U[5] + U[2] * U[6] + U[3] * U[7]
    else:
        BB = np.zeros_like(D)
        SB = np.zeros_like(D)
    f0, valid = oracle.pressure_function_points(system, gamma, U, np.zeros_like(D))
    f0 = np.where(valid & (f0 > 0), f0, 1e-300 * D)
    return np.stack([np.log(tau / D), np.log1p(np.sqrt(S2) / D), np.log1p(BB / D),
                     SB / (np.sqrt(S2) * np.sqrt(BB) + 1e-30), np.log(f0 / D)])


def silu(a):
    return a / (1.0 + np.exp(-a))


def dsilu(a):
    s = 1.0 / (1.0 + np.exp(-a))
    return s * (1.0 + a * (1.0 - s))


def normalise(params, x, t=None):
    p = np.asarray(params, dtype=np.float64)
    xn = (np.asarray(x, dtype=np.float64) - p[O_MU:O_MU + IN, None]) / p[O_SD:O_SD + IN, None]
    if t is None:
        return xn
    return xn, (np.asarray(t, dtype=np.float64) - p[O_YMU]) / p[O_YSD]


def forward_normalised(params, xn):
    """xn[5][B] -> y[B] (normalised output) and the activations."""
    W1, b1, W2, b2, W3, b3 = unpack(params)
    a1 = W1 @ xn + b1[:, None]
    h1 = silu(a1)
    a2 = W2 @ h1 + b2[:, None]
    h2 = silu(a2)
    y = W3 @ h2 + b3
    return y, (a1, h1, a2, h2)


def predict(params, x):
    """Raw features -> predicted ln(p/D)."""
    p = np.asarray(params, dtype=np.float64)
    y, _ = forward_normalised(p, normalise(p, x))
    return y * p[O_YSD] + p[O_YMU]


def loss_and_grad(params, x, t):
    """Mean squared error in normalised units and its gradient w.r.t. the
    4609 weights (back-propagation)."""
    p = np.asarray(params, dtype=np.float64)
    xn, tn = normalise(p, x, t)
    B = xn.shape[1]
    W1, b1, W2, b2, W3, b3 = unpack(p)
    y, (a1, h1, a2, h2) = forward_normalised(p, xn)
    r = y - tn
    loss = np.mean(r * r)
    dy = 2.0 * r / B
    g = np.zeros(NW)
    g[O_W3:O_B3] = h2 @ dy
    g[O_B3] = dy.sum()
    da2 = (W3[:, None] * dy[None, :]) * dsilu(a2)
    g[O_W2:O_B2] = (da2 @ h1.T).ravel()
    g[O_B2:O_W3] = da2.sum(axis=1)
    da1 = (W2.T @ da2) * dsilu(a1)
    g[O_W1:O_B1] = (da1 @ xn.T).ravel()
    g[O_B1:O_W2] = da1.sum(axis=1)
    return loss, g


def loss(params, x, t):
    p = np.asarray(params, dtype=np.float64)
    xn, tn = normalise(p, x, t)
    y, _ = forward_normalised(p, xn)
    return np.mean((y - tn) ** 2)


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of the weights (normalisation entries untouched).
    Returns new (params, m, v); step is the 1-based step count."""
    p = np.array(params, dtype=np.float64)
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    p[:NW] -= lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v
