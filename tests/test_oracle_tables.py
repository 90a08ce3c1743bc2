"""Pins of the oracle's GLL tables against textbook facts (not against itself).

Nodal basis: Lagrange polynomials on Gauss-Legendre-Lobatto nodes (algorithm
section of the paper); D_il = ell_l'(x_i) (eq. for D^{1bar}); diagonal GLL
mass matrix (Appendix B).
"""
import math

import numpy as np
import pytest


# Closed-form GLL nodes/weights from quadrature tables (Abramowitz & Stegun 25.4.32).
KNOWN = {
    1: ([-1.0, 1.0], [1.0, 1.0]),
    2: ([-1.0, 0.0, 1.0], [1 / 3, 4 / 3, 1 / 3]),
    3: ([-1.0, -1 / math.sqrt(5), 1 / math.sqrt(5), 1.0], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    4: ([-1.0, -math.sqrt(3 / 7), 0.0, math.sqrt(3 / 7), 1.0], [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
}


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_gll_closed_forms(ora, N):
    x, w = ora.gll(N)
    xk, wk = KNOWN[N]
    assert np.allclose(x, xk, atol=1e-15, rtol=0)
    assert np.allclose(w, wk, atol=1e-15, rtol=0)


@pytest.mark.parametrize("N", range(1, 8))
def test_gll_quadrature_exactness(ora, N):
    x, w = ora.gll(N)
    # GLL with N+1 points integrates polynomials of degree <= 2N-1 exactly
    for m in range(2 * N):
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(np.dot(w, x ** m) - exact) < 1e-14
    # ... and not degree 2N (the rule's defect), which pins the node count
    assert abs(np.dot(w, x ** (2 * N)) - 2.0 / (2 * N + 1)) > 1e-6
    assert abs(w[0] - 2.0 / (N * (N + 1))) < 1e-15
    assert np.allclose(x, -x[::-1], atol=1e-15)


@pytest.mark.parametrize("N", range(1, 8))
def test_diff_matrix_against_lagrange_derivatives(ora, N):
    """D_il = ell_l'(x_i) computed independently from numpy's polynomial class."""
    x, _ = ora.gll(N)
    D = ora.diff_matrix(N)
    for l in range(N + 1):
        others = np.delete(x, l)
        poly = np.polynomial.Polynomial.fromroots(others)
        poly = poly / poly(x[l])
        dpoly = poly.deriv()
        assert np.allclose(D[:, l], dpoly(x), atol=2e-13, rtol=0)


@pytest.mark.parametrize("N", range(1, 8))
def test_diff_matrix_exact_on_polynomials_and_sbp(ora, N):
    x, w = ora.gll(N)
    D = ora.diff_matrix(N)
    for m in range(N + 1):
        d_exact = m * x ** (m - 1) if m > 0 else np.zeros_like(x)
        assert np.abs(D @ x ** m - d_exact).max() < 1e-12
    # summation-by-parts: W D + (W D)^T = diag(-1, 0, ..., 0, 1)
    Q = np.diag(w) @ D
    B = np.zeros((N + 1, N + 1))
    B[0, 0], B[N, N] = -1.0, 1.0
    assert np.abs(Q + Q.T - B).max() < 1e-14


def test_legendre_values(ora):
    # P_N(1) = 1, P_N(-1) = (-1)^N, P_2(x) = (3x^2-1)/2
    for N in range(8):
        assert abs(ora.legendre(N, 1.0) - 1.0) < 1e-15
        assert abs(ora.legendre(N, -1.0) - (-1.0) ** N) < 1e-15
    assert abs(ora.legendre(2, 0.3) - (3 * 0.09 - 1) / 2) < 1e-15


@pytest.mark.parametrize("nf,nt", [(3, 5), (4, 8), (8, 8), (5, 3)])
def test_lagrange_matrix(ora, nf, nt):
    xf, _ = ora.gll(nf - 1)
    yt, _ = ora.gll(nt - 1)
    I = ora.lagrange_matrix(xf, yt)
    # reproduces every polynomial of degree <= nf-1 when nt >= nf
    if nt >= nf:
        for m in range(nf):
            assert np.abs(I @ xf ** m - yt ** m).max() < 1e-13
    # partition of unity
    assert np.abs(I.sum(1) - 1.0).max() < 1e-13
    # identity on its own nodes
    assert np.abs(ora.lagrange_matrix(xf, xf) - np.eye(nf)).max() < 1e-15
