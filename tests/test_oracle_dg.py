"""Pins of the oracle's DG operator and stepper against what the method fixes.

* free-stream preservation: a constant state has a zero right-hand side;
* the strong form (eq. 411) equals the independently coded weak form (eq. 4
  evaluated with GLL quadrature) -- this fixes the lift's scale and sign;
* discrete conservation: the GLL-weighted sum of the RHS vanishes on a
  periodic mesh (the numerical flux is single valued on interfaces);
* spatial convergence of the RHS to the exact time derivative of the
  advected smooth flow at order >= N;
* SSP-RK3: linear amplification factor 1 + z + z^2/2 + z^3/6 and third-order
  temporal convergence.
"""
import math

import numpy as np
import pytest

from paper_1609_00098_amd import synth

NE, SR, MHD = 0, 1, 2
NV = {NE: 5, SR: 5, MHD: 9}


def _state(ora, system, m, seed=3):
    xyz = ora.node_coords(m)
    lo = np.array(m.lo[:])
    hi = np.array(m.hi[:])
    unit = (xyz - lo[:, None]) / (hi - lo)[:, None]
    g = m.gamma
    if system == MHD:
        prim = synth.fourier_random_prims(unit, seed=seed, w_max=3.0, rho_range=(0.5, 2.0), p_range=(0.1, 10.0))
        rng = np.random.default_rng(seed)
        mag = np.zeros((4, prim.shape[1]))
        for c in range(4):
            k = rng.integers(1, 3, size=3)
            mag[c] = 0.3 * np.sin(2 * np.pi * (k @ unit) + rng.uniform(0, 6))
        mag[0] += 1.0
        return ora.prim2cons(MHD, g, prim, mag)
    prim = synth.fourier_random_prims(unit, seed=seed, w_max=5.0 if system == SR else 1.5)
    if system == NE:
        prim[1:4] *= 2.0
    return ora.prim2cons(system, g, prim)


MESHES = [
    (NE, (2, 3, 2), (3, 3, 3)),
    (SR, (3, 2, 2), (4, 4, 4)),
    (MHD, (2, 2, 3), (2, 2, 2)),
    (SR, (2, 2, 2), (2, 5, 3)),
    (SR, (5, 1, 1), (3, 0, 0)),
]


def _mesh(ora, system, nel, deg):
    return ora.mesh(system, nel, deg, 4.0 / 3.0 if system else 1.4, lo=(-0.3, 0.1, 0.0), hi=(0.7, 1.6, 2.0),
                    kappa=0.5)


@pytest.mark.parametrize("system,nel,deg", MESHES)
def test_free_stream(ora, system, nel, deg):
    m = _mesh(ora, system, nel, deg)
    n = ora.num_nodes(m)
    prim = np.tile(np.array([[1.3], [0.3], [-0.2], [0.25], [0.7]]), (1, n))
    mag = np.tile(np.array([[0.4], [-0.3], [0.2], [0.0]]), (1, n))
    U = ora.prim2cons(system, m.gamma, prim, mag if system == MHD else None)
    dU, _, nf = ora.rhs(m, U)
    assert nf == 0
    assert np.abs(dU).max() < 1e-12


@pytest.mark.parametrize("system,nel,deg", MESHES)
def test_strong_equals_weak(ora, system, nel, deg):
    m = _mesh(ora, system, nel, deg)
    U = _state(ora, system, m)
    s, _, nf = ora.rhs(m, U)
    w = ora.rhs_weak(m, U)
    assert nf == 0
    for v in range(NV[system]):
        scale = np.abs(s[v]).max()
        assert np.abs(s[v] - w[v]).max() <= 1e-12 * scale


@pytest.mark.parametrize("system,nel,deg", MESHES)
def test_discrete_conservation(ora, system, nel, deg):
    m = _mesh(ora, system, nel, deg)
    U = _state(ora, system, m)
    dU, _, _ = ora.rhs(m, U)
    tot = ora.integrate(m, dU)
    absint = ora.integrate(m, np.abs(dU))
    if system == MHD:
        # the cleaning scalar is damped by its source, -kappa Phi
        tot[8] -= ora.integrate(m, -m.kappa * U[8:9])[0]
    assert np.all(np.abs(tot) <= 1e-13 * absint.max())


def _smooth_flow_exact_rhs(xyz, g, v, A=0.2, k=2 * math.pi):
    """dU/dt for the advected wave (constant v, p = 1): -(v.grad rho) dU/drho."""
    phase = xyz[0] + xyz[1] + xyz[2]
    drho = A * k * np.cos(k * phase) * sum(v)
    W = 1.0 / math.sqrt(1.0 - sum(c * c for c in v))
    out = np.zeros((5, xyz.shape[1]))
    out[0] = -drho * W
    for i in range(3):
        out[1 + i] = -drho * W * W * v[i]
    out[4] = -drho * (W * W - W)
    return out


@pytest.mark.parametrize("N", [2, 3])
def test_rhs_converges_to_exact_time_derivative(ora, N):
    g = 5.0 / 3.0
    v = (0.2, 0.2, 0.2)
    errs = []
    for K in (2, 4, 8):
        m = ora.mesh(SR, (K, K, K), N, g)
        xyz = ora.node_coords(m)
        U = ora.prim2cons(SR, g, synth.smooth_flow(xyz, 0.0, 0.2, 2 * math.pi, v))
        dU, _, _ = ora.rhs(m, U)
        errs.append(np.abs(dU - _smooth_flow_exact_rhs(xyz, g, v)).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert rates[-1] > N - 0.3, (errs, rates)


def test_rk3_amplification_factor(ora):
    """For L(y) = lambda y the three Shu-Osher stages give R(z) y0 with
    R(z) = 1 + z + z^2/2 + z^3/6, the third-order Taylor polynomial."""
    lam = np.array([-1.0, -0.3, 0.5, -2.0])
    dt = 0.37
    y0 = np.array([1.0, 2.0, -0.5, 3.0])
    y1 = ora.rk3_combine(1, dt, y0, y0, lam * y0)
    y2 = ora.rk3_combine(2, dt, y0, y1, lam * y1)
    y3 = ora.rk3_combine(3, dt, y0, y2, lam * y2)
    z = lam * dt
    assert np.allclose(y3, (1 + z + z * z / 2 + z ** 3 / 6) * y0, rtol=1e-15, atol=1e-15)
    with pytest.raises(ValueError):
        ora.rk3_combine(4, dt, y0, y0, y0)


def test_rk3_third_order_in_time(ora):
    g = 5.0 / 3.0
    m = ora.mesh(SR, (4, 1, 1), (4, 0, 0), g)
    xyz = ora.node_coords(m)
    U0 = ora.prim2cons(SR, g, synth.smooth_flow(xyz, 0.0, 0.2, 2 * math.pi, (0.2, 0, 0), active=(True, False, False)))
    T = 0.08
    ref, _ = ora.evolve(m, U0, T / 64, 64)
    errs = []
    for nst in (4, 8):
        u, _ = ora.evolve(m, U0, T / nst, nst)
        errs.append(np.abs(u - ref).max())
    assert 2.6 < math.log2(errs[0] / errs[1]) < 3.4


@pytest.mark.parametrize("system", [NE, SR])
def test_step_conserves_totals(ora, system):
    m = _mesh(ora, system, (3, 2, 2), (3, 3, 3))
    U = _state(ora, system, m)
    before = ora.integrate(m, U)
    U1, nf = ora.step(m, U, 1e-5)
    after = ora.integrate(m, U1)
    assert nf == 0
    assert np.all(np.abs(after - before) <= 1e-13 * np.abs(before).max())
    assert np.abs(U1 - U).max() > 1e-6
