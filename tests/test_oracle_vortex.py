"""Pins of the oracle's analytic boundary condition with the isentropic
vortex (eq. isen_vortex) and of the vortex itself:

* the oracle's vortex equals the independently written generator (two
  codings of the printed formula; the generator is also the initial data);
* the vortex solves the Euler equations: with the exact solution as both the
  state and the exterior boundary state, the DG operator approaches the
  exact time derivative (central difference in t) at the element order,
  boundary nodes included -- a wrong exterior state or orientation would
  leave an O(1) error at the boundary;
* the stage times: one RK3 step from the exact state stays within the
  scheme's error of the exact state at t + dt;
* the polytropic equation of state p = rho^gamma (the vortex test's
  adiabatic one) gives p from the density alone, independent of the energy;
* the scheme reproduces tab:IsenVortexConvergence (K = 8, N_C = 2 by
  default; K = 8, N_C = 3 and K = 16, N_C = 2 with DGMI_SLOW=1).
"""
import json
import math
import os

import numpy as np
import pytest

from paper_1609_00098_amd import synth

NE = 0
G = 1.4
PAR = (5.0, 4.0, 4.0, 1.0, 1.0, 0.0)
GOLD = os.path.join(os.path.dirname(__file__), "golden")
SLOW = os.environ.get("DGMI_SLOW") == "1"


def _mesh(ora, K, N, time=0.0, eos="polytropic"):
    return ora.mesh(NE, (K, K, 1), N, G, lo=(0, 0, 0), hi=(10, 10, 1), vortex=PAR, time=time,
                    bc={0: "vortex", 1: "vortex", 2: "vortex"}, eos=eos)


def test_vortex_formula_two_codings(ora):
    xyz = np.random.default_rng(0).uniform(0, 10, size=(3, 1000))
    for t in (0.0, 0.7, 2.0):
        a = ora.isentropic_vortex(G, PAR, xyz, t)
        b = synth.isentropic_vortex(xyz, t)
        assert np.allclose(a, b, rtol=1e-14, atol=1e-15)
    # far from the centre: the uniform flow with rho = p = 1
    far = ora.isentropic_vortex(G, PAR, np.array([[9.9], [0.1], [0.5]]), 0.0)
    assert np.allclose(far[:, 0], [1.0, 1.0, 1.0, 0.0, 1.0], atol=1e-6)


def test_polytropic_pressure(ora):
    m = _mesh(ora, 2, 2)
    n = ora.num_nodes(m)
    rng = np.random.default_rng(4)
    prim = np.stack([rng.uniform(0.5, 2, n), rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(-1, 1, n),
                     np.zeros(n)])
    prim[4] = prim[0] ** G
    U = ora.prim2cons(NE, G, prim)
    U[4] += rng.uniform(0, 1, n)  # the energy does not enter the pressure
    _, P, nf = ora.rhs(m, U)
    assert nf == 0
    assert np.allclose(P[4], prim[0] ** G, rtol=1e-15) and np.allclose(P[:4], prim[:4], rtol=1e-14)
    mi = _mesh(ora, 2, 2, eos="ideal")
    _, Pi, _ = ora.rhs(mi, U)
    assert np.abs(Pi[4] - P[4]).max() > 0.1
    with pytest.raises(ValueError):
        ora.rhs(ora.mesh(1, (2, 2, 2), 2, 4.0 / 3.0, eos="polytropic"), np.ones((5, 216)))


def _dudt_exact(ora, xyz, t, h=1e-5):
    up = ora.prim2cons(NE, G, ora.isentropic_vortex(G, PAR, xyz, t + h))
    um = ora.prim2cons(NE, G, ora.isentropic_vortex(G, PAR, xyz, t - h))
    return (up - um) / (2 * h)


def test_operator_with_analytic_boundary_is_consistent(ora):
    errs = []
    t = 0.3
    N = 4
    for K in (4, 8):
        m = _mesh(ora, K, N, time=t)
        xyz = ora.node_coords(m)
        U = ora.prim2cons(NE, G, ora.isentropic_vortex(G, PAR, xyz, t))
        dU, _, nf = ora.rhs(m, U)
        assert nf == 0
        ex = _dudt_exact(ora, xyz, t)
        edge = (xyz[0] < 1e-12) | (xyz[0] > 10 - 1e-12) | (xyz[1] < 1e-12) | (xyz[1] > 10 - 1e-12)
        assert edge.sum() > 0
        errs.append((np.abs(dU - ex).max(), np.abs(dU - ex)[:, edge].max()))
    # whole domain and boundary nodes alike converge at about order N
    assert math.log2(errs[0][0] / errs[1][0]) > N - 1.0, errs
    assert errs[1][1] < 1e-2 * np.abs(ex).max(), errs
    # a wrong exterior (the state at rest) leaves an O(1) error at the boundary
    m_bad = ora.mesh(NE, (8, 8, 1), N, G, lo=(0, 0, 0), hi=(10, 10, 1), time=t,
                     bc={0: ((1, 0, 0, 0, 1), (1, 0, 0, 0, 1)), 1: ((1, 0, 0, 0, 1), (1, 0, 0, 0, 1))})
    dUb, _, _ = ora.rhs(m_bad, U)
    assert np.abs(dUb - ex)[:, edge].max() > 1e2 * errs[1][1]


def test_one_step_tracks_the_exact_solution(ora):
    t, dt = 0.5, 1e-3
    m = _mesh(ora, 8, 3, time=t)
    xyz = ora.node_coords(m)
    U = ora.prim2cons(NE, G, ora.isentropic_vortex(G, PAR, xyz, t))
    U1, nf = ora.step(m, U, dt)
    assert nf == 0
    ex = ora.prim2cons(NE, G, ora.isentropic_vortex(G, PAR, xyz, t + dt))
    dU, _, _ = ora.rhs(m, U)
    # the step error is dt times the operator's spatial error (plus O(dt^4))
    spatial = np.abs(dU - _dudt_exact(ora, xyz, t)).max()
    assert np.abs(U1 - ex).max() <= 1.5 * dt * spatial + 1e-12


def _vortex_error(ora, K, NC):
    m = _mesh(ora, K, NC - 1)
    xyz = ora.node_coords(m)
    U0 = ora.prim2cons(NE, G, ora.isentropic_vortex(G, PAR, xyz, 0.0))
    U1, nf = ora.evolve(m, U0, 1e-4, 20000)
    assert nf == 0
    return ora.l1_error(m, ora.prim2cons(NE, G, ora.isentropic_vortex(G, PAR, xyz, 2.0)), U1)


@pytest.mark.parametrize("K,NC", [(8, 2)] + ([(8, 3), (16, 2)] if SLOW else []))
def test_isentropic_vortex_table(ora, K, NC):
    """tab:IsenVortexConvergence within 1% of the printed value.  Readings:
    the adiabatic equation of state P = rho^gamma of the test's text is the
    evolution's equation of state (with the ideal gas the errors come out
    up to 2.2 times the printed ones at high order); analytic boundaries on
    every outer face, z included (with one element along z those faces
    pull the state towards the exact one; periodic z gives errors 1.3-1.9
    times larger)."""
    gold = json.load(open(os.path.join(GOLD, "isentropic_vortex_table.json")))
    ref = gold["rows_NC"][str(NC)][gold["columns_K"].index(K)]
    err = _vortex_error(ora, K, NC)
    assert abs(err - ref) <= 0.01 * ref, (err, ref)
