"""Pins of the oracle's time-step helpers (CFL scaling of the section on
initial data, boundary conditions and time steppers) and of its third-order
Adams-Bashforth stepper:

* the largest characteristic speed equals closed forms: the sound speed at
  rest (Newtonian and relativistic), |v_d| + c_s for a uniform Newtonian
  flow, the light speed for SRMHD (cleaning);
* the smallest GLL node spacing equals the closed-form node gaps
  (N = 1: dx; N = 2: dx/2; N = 3: (1 - 1/sqrt5) dx/2; N = 4:
  (1 - sqrt(3/7)) dx/2);
* AB3: its first two steps are the SSP-RK3 steps that start its history;
  it conserves the discrete totals; its temporal error falls at order 3.
"""
import math

import numpy as np
import pytest

from paper_1609_00098_amd import synth

NE, SR, MHD = 0, 1, 2


def _uniform(ora, system, m, prim5, mag=None):
    n = ora.num_nodes(m)
    prim = np.tile(np.asarray(prim5, dtype=float)[:, None], (1, n))
    mg = None if mag is None else np.tile(np.asarray(mag, dtype=float)[:, None], (1, n))
    return ora.prim2cons(system, m.gamma, prim, mg)


def test_max_char_speed_closed_forms(ora):
    g = 1.4
    m = ora.mesh(NE, (2, 2, 2), 2, g)
    U = _uniform(ora, NE, m, (1.3, 0.0, 0.0, 0.0, 0.7))
    assert abs(ora.max_char_speed(m, U) - math.sqrt(g * 0.7 / 1.3)) < 1e-15
    U = _uniform(ora, NE, m, (1.3, 0.3, -0.5, 0.1, 0.7))
    assert abs(ora.max_char_speed(m, U) - (0.5 + math.sqrt(g * 0.7 / 1.3))) < 1e-15
    gr = 4.0 / 3.0
    ms = ora.mesh(SR, (2, 2, 2), 2, gr)
    U = _uniform(ora, SR, ms, (1.3, 0.0, 0.0, 0.0, 0.7))
    h = 1 + gr / (gr - 1) * 0.7 / 1.3
    assert abs(ora.max_char_speed(ms, U) - math.sqrt(gr * 0.7 / (1.3 * h))) < 1e-15
    mm = ora.mesh(MHD, (2, 2, 2), 2, gr)
    U = _uniform(ora, MHD, mm, (1.3, 0.2, 0.0, 0.0, 0.7), (0.5, 0.1, 0.0, 0.0))
    assert ora.max_char_speed(mm, U) == 1.0


def test_min_node_spacing_closed_forms(ora):
    dx = 0.25
    gaps = {1: 1.0, 2: 0.5, 3: 0.5 * (1 - 1 / math.sqrt(5)), 4: 0.5 * (1 - math.sqrt(3 / 7))}
    for N, gap in gaps.items():
        m = ora.mesh(NE, (4, 2, 8), N, 1.4, hi=(1.0, 1.0, 2.0))  # dx = 0.25 in x and z, 0.5 in y
        assert abs(ora.min_node_spacing(m) - gap * dx) < 1e-15
    m = ora.mesh(NE, (4, 2, 8), 3, 1.4, hi=(1.0, 1.0, 2.0))
    U = _uniform(ora, NE, m, (1.0, 0.0, 0.0, 0.0, 1.0))
    assert abs(ora.stable_dt(m, U, 0.3) - 0.3 * gaps[3] * dx / math.sqrt(1.4)) < 1e-16


def _wave(ora, m, g=5.0 / 3.0):
    xyz = ora.node_coords(m)
    return ora.prim2cons(SR, g, synth.smooth_flow(xyz, 0.0, 0.2, 2 * math.pi, (0.2, 0, 0),
                                                  active=(True, False, False)))


def test_ab3_starts_with_rk3_steps_and_conserves(ora):
    g = 5.0 / 3.0
    m = ora.mesh(SR, (4, 1, 1), (4, 0, 0), g)
    U0 = _wave(ora, m)
    a, _ = ora.evolve_ab3(m, U0, 1e-3, 2)
    b, _ = ora.evolve(m, U0, 1e-3, 2)
    assert np.array_equal(a, b)
    m3 = ora.mesh(SR, (3, 2, 2), 3, 4.0 / 3.0)
    xyz = ora.node_coords(m3)
    U = ora.prim2cons(SR, m3.gamma, synth.fourier_random_prims(xyz, seed=5, w_max=2.0, rho_range=(0.5, 2),
                                                               p_range=(0.5, 2)))
    before = ora.integrate(m3, U)
    U1, nf = ora.evolve_ab3(m3, U, 1e-4, 6)
    assert nf == 0
    after = ora.integrate(m3, U1)
    assert np.all(np.abs(after - before) <= 1e-13 * np.abs(before).max())


def test_ab3_third_order_in_time(ora):
    g = 5.0 / 3.0
    m = ora.mesh(SR, (4, 1, 1), (4, 0, 0), g)
    U0 = _wave(ora, m)
    T = 0.08
    ref, _ = ora.evolve(m, U0, T / 256, 256)
    errs = []
    for nst in (16, 32, 64):
        u, nf = ora.evolve_ab3(m, U0, T / nst, nst)
        assert nf == 0
        errs.append(np.abs(u - ref).max())
    for a, b in zip(errs, errs[1:]):
        assert 2.6 < math.log2(a / b) < 3.4, errs
