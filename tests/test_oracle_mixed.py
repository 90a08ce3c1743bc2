"""Pins of the oracle's mixed-degree operator (mortars between elements of
unequal degree; the paper defers such coupling, so the reading is: mortar of
the larger degree, interpolated primitives on the lower side, and a face
projection weighted by the mortar's GLL rule).

* equal degrees reduce bit for bit to the uniform-degree operator;
* free stream: a constant state has a zero right-hand side;
* discrete conservation with every element's own GLL rule (the mortar flux
  is single valued and both sides integrate it with the mortar rule);
* a pressure field that is continuous and bilinear, at rest, has no surface
  term on any face, conforming or not, so every element's right-hand side is
  the exact pressure gradient (fixes interpolation/projection orientation);
* an element whose primitives are polynomials of its own degree gives the
  same mortar states as the conforming operator of the higher degree;
* spatial convergence of the right-hand side on a checkerboard of degrees.
"""
import math

import numpy as np
import pytest

from paper_1609_00098_amd import synth

NE, SR, MHD = 0, 1, 2
NV = {NE: 5, SR: 5, MHD: 9}


def _mesh(ora, system, nel, deg=2):
    return ora.mesh(system, nel, deg, 4.0 / 3.0 if system else 1.4, lo=(-0.3, 0.1, 0.0), hi=(0.7, 1.6, 2.0),
                    kappa=0.5)


def _state(ora, system, m, deg, seed=3):
    xyz = ora.mixed_node_coords(m, deg)
    lo = np.array(m.lo[:])
    hi = np.array(m.hi[:])
    unit = (xyz - lo[:, None]) / (hi - lo)[:, None]
    if system == MHD:
        prim = synth.fourier_random_prims(unit, seed=seed, w_max=3.0, rho_range=(0.5, 2.0), p_range=(0.1, 10.0))
        rng = np.random.default_rng(seed)
        mag = np.zeros((4, prim.shape[1]))
        for c in range(4):
            k = rng.integers(1, 3, size=3)
            mag[c] = 0.3 * np.sin(2 * np.pi * (k @ unit) + rng.uniform(0, 6))
        mag[0] += 1.0
        return ora.prim2cons(MHD, m.gamma, prim, mag)
    prim = synth.fourier_random_prims(unit, seed=seed, w_max=5.0 if system == SR else 1.5)
    return ora.prim2cons(system, m.gamma, prim)


@pytest.mark.parametrize("system,N", [(NE, 3), (SR, 4), (MHD, 2), (SR, 1)])
def test_equal_degrees_reduce_to_uniform_operator(ora, system, N):
    m = _mesh(ora, system, (3, 2, 2), N)
    deg = np.full(12, N, np.int32)
    U = _state(ora, system, m, deg)
    a, pa, nfa = ora.rhs(m, U)
    b, pb, nfb = ora.rhs_mixed(m, deg, U)
    assert nfa == nfb == 0
    assert np.array_equal(a, b)
    assert np.array_equal(pa, pb)


DEGS = {
    "checker23": lambda ne: np.array([2 + (e % 2) for e in range(ne)], np.int32),
    "random27": lambda ne: synth.mixed_degrees(ne, seed=1610),
    "random15": lambda ne: synth.mixed_degrees(ne, seed=7, lo=1, hi=5),
}


@pytest.mark.parametrize("system", [NE, SR, MHD])
@pytest.mark.parametrize("degs", sorted(DEGS))
def test_mixed_free_stream(ora, system, degs):
    m = _mesh(ora, system, (3, 3, 2))
    deg = DEGS[degs](18)
    n = ora.mixed_num_nodes(deg)
    prim = np.tile(np.array([[1.3], [0.3], [-0.2], [0.25], [0.7]]), (1, n))
    mag = np.tile(np.array([[0.4], [-0.3], [0.2], [0.0]]), (1, n))
    U = ora.prim2cons(system, m.gamma, prim, mag if system == MHD else None)
    dU, _, nf = ora.rhs_mixed(m, deg, U)
    assert nf == 0
    # rounding of the differentiation matrix grows like N^2 times 2/dx
    dxmin = min((m.hi[d] - m.lo[d]) / (3, 3, 2)[d] for d in range(3))
    assert np.abs(dU).max() < 2e-14 * deg.max() ** 2 * (2.0 / dxmin) * np.abs(U).max()


@pytest.mark.parametrize("system", [NE, SR, MHD])
@pytest.mark.parametrize("degs", sorted(DEGS))
def test_mixed_discrete_conservation(ora, system, degs):
    m = _mesh(ora, system, (3, 3, 2))
    deg = DEGS[degs](18)
    U = _state(ora, system, m, deg)
    dU, _, nf = ora.rhs_mixed(m, deg, U)
    assert nf == 0
    tot = ora.mixed_integrate(m, deg, dU)
    absint = ora.mixed_integrate(m, deg, np.abs(dU))
    if system == MHD:
        tot[8] -= ora.mixed_integrate(m, deg, -m.kappa * U[8:9])[0]
    assert np.all(np.abs(tot) <= 1e-13 * absint.max())


def _bilinear_p(xyz):
    x, y, z = xyz
    return 1.0 + 0.1 * x + 0.05 * y - 0.07 * z + 0.02 * x * y - 0.03 * y * z + 0.04 * x * z


@pytest.mark.parametrize("centre,around", [(2, (3, 4, 5, 3, 4, 6)), (5, (2, 3, 4, 2, 3, 2)), (3, (3, 3, 3, 3, 3, 3))])
def test_continuous_bilinear_pressure_has_no_surface_term(ora, centre, around):
    """Fluid at rest with constant density and a pressure that is continuous
    and of degree one in each coordinate: the flux is p n with no jump, so
    the right-hand side of the centre element of a 3x3x3 mesh (and of its six
    face neighbours, at their shared faces) is (0, -grad p, 0)."""
    m = ora.mesh(NE, (3, 3, 3), 2, 1.4, lo=(-1.0, -1.0, -1.0), hi=(2.0, 2.0, 2.0))
    deg = np.full(27, 3, np.int32)
    c = 13
    deg[c] = centre
    nb = [c - 1, c + 1, c - 3, c + 3, c - 9, c + 9]
    for e, d in zip(nb, around):
        deg[e] = d
    xyz = ora.mixed_node_coords(m, deg)
    n = xyz.shape[1]
    prim = np.zeros((5, n))
    prim[0] = 1.0
    prim[4] = _bilinear_p(xyz)
    U = ora.prim2cons(NE, m.gamma, prim)
    dU, _, nf = ora.rhs_mixed(m, deg, U)
    assert nf == 0
    x, y, z = xyz
    grad = np.stack([0.1 + 0.02 * y + 0.04 * z, 0.05 + 0.02 * x - 0.03 * z, -0.07 - 0.03 * y + 0.04 * x])
    off = np.concatenate([[0], np.cumsum((deg.astype(np.int64) + 1) ** 3)])
    sl = slice(off[c], off[c + 1])
    assert np.abs(dU[0, sl]).max() < 1e-13
    assert np.abs(dU[4, sl]).max() < 1e-13
    assert np.abs(dU[1:4, sl] + grad[:, sl]).max() < 1e-13
    # the neighbours' nodes on the faces they share with the centre
    for e in nb:
        s = slice(off[e], off[e + 1])
        near = np.all(np.abs(xyz[:, s] - np.clip(xyz[:, s], 0.0, 1.0)) < 1e-12, axis=0)
        assert near.sum() == (deg[e] + 1) ** 2
        assert np.abs(dU[1:4, s][:, near] + grad[:, s][:, near]).max() < 1e-13


@pytest.mark.parametrize("system", [SR, MHD])
def test_polynomial_element_matches_conforming_operator(ora, system):
    """Centre element of degree 2 among degree-3 elements, with rho, W v, p
    (and B, Phi) polynomials of degree <= 2 in each coordinate inside it: its interpolated mortar states are the degree-3 face values, so every
    other element's right-hand side equals the uniform degree-3 operator's."""
    m3 = _mesh(ora, system, (3, 3, 3), 3)
    deg = np.full(27, 3, np.int32)
    c = 13
    deg[c] = 2
    g = m3.gamma

    def fields(xyz, in_centre):
        unit = (xyz - np.array(m3.lo[:])[:, None]) / (np.array(m3.hi[:]) - np.array(m3.lo[:]))[:, None]
        prim = synth.fourier_random_prims(unit, seed=5, w_max=2.0, rho_range=(0.5, 2.0), p_range=(0.5, 5.0))
        mag = np.zeros((4, xyz.shape[1]))
        mag[0], mag[1], mag[2] = 0.8, -0.3 + 0.1 * unit[0], 0.2 * unit[1]
        x, y, z = unit[:, in_centre]
        q = 1.0 + 0.3 * x - 0.2 * y * y + 0.1 * x * y * z + 0.05 * z * z * x
        prim[0, in_centre] = q
        # the mortar interpolates the spatial four-velocity u = W v
        u = np.stack([0.2 * q - 0.1, 0.1 * x * y, -0.15 * z * z])
        prim[1:4, in_centre] = u / np.sqrt(1.0 + (u * u).sum(0))
        prim[4, in_centre] = 0.5 + x * z
        mag[1, in_centre] = 0.3 * x * y
        mag[3, in_centre] = 0.05 * y * z
        return prim, (mag if system == MHD else None)

    def centre_mask(mesh, dg):
        off = np.concatenate([[0], np.cumsum((dg.astype(np.int64) + 1) ** 3)])
        msk = np.zeros(off[-1], bool)
        msk[off[c]:off[c + 1]] = True
        return msk

    xm = ora.mixed_node_coords(m3, deg)
    mm = centre_mask(m3, deg)
    Um = ora.prim2cons(system, g, *fields(xm, mm))
    dm, _, nf1 = ora.rhs_mixed(m3, deg, Um)
    d3 = np.full(27, 3, np.int32)
    xu = ora.node_coords(m3)
    mu = centre_mask(m3, d3)
    Uu = ora.prim2cons(system, g, *fields(xu, mu))
    du, _, nf2 = ora.rhs(m3, Uu)
    assert nf1 == nf2 == 0
    keep_m, keep_u = ~mm, ~mu
    scale = np.abs(du[:, keep_u]).max(axis=1, keepdims=True)
    err = np.abs(dm[:, keep_m] - du[:, keep_u]) / scale
    assert err.max() < 1e-11, err.max()


def _smooth_flow_exact_rhs(xyz, v, A=0.2, k=2 * math.pi):
    phase = xyz[0] + xyz[1] + xyz[2]
    drho = A * k * np.cos(k * phase) * sum(v)
    W = 1.0 / math.sqrt(1.0 - sum(c * c for c in v))
    out = np.zeros((5, xyz.shape[1]))
    out[0] = -drho * W
    for i in range(3):
        out[1 + i] = -drho * W * W * v[i]
    out[4] = -drho * (W * W - W)
    return out


@pytest.mark.parametrize("lo,hi", [(2, 3), (3, 4)])
def test_mixed_rhs_converges(ora, lo, hi):
    """Checkerboard of degrees lo/hi: the RHS error against the exact time
    derivative of the advected wave falls at order lo (max and GLL L2 norms,
    K = 8 -> 16 elements per direction)."""
    g = 5.0 / 3.0
    v = (0.2, 0.2, 0.2)
    emax, el2 = [], []
    for K in (4, 8, 16):
        m = ora.mesh(SR, (K, K, K), 2, g)
        e = np.arange(K ** 3)
        deg = np.where(((e % K) + (e // K) % K + e // (K * K)) % 2 == 0, lo, hi).astype(np.int32)
        xyz = ora.mixed_node_coords(m, deg)
        U = ora.prim2cons(SR, g, synth.smooth_flow(xyz, 0.0, 0.2, 2 * math.pi, v))
        dU, _, nf = ora.rhs_mixed(m, deg, U)
        assert nf == 0
        err = dU - _smooth_flow_exact_rhs(xyz, v)
        emax.append(np.abs(err).max())
        el2.append(math.sqrt(ora.mixed_integrate(m, deg, err * err).sum()))
    rmax = math.log2(emax[1] / emax[2])
    rl2 = math.log2(el2[1] / el2[2])
    assert rmax > lo - 0.2 and rl2 > lo - 0.2, (emax, el2)


@pytest.mark.parametrize("system", [NE, SR])
def test_mixed_step_conserves_totals(ora, system):
    m = _mesh(ora, system, (3, 2, 2))
    deg = synth.mixed_degrees(12, seed=1610)
    U = _state(ora, system, m, deg)
    before = ora.mixed_integrate(m, deg, U)
    U1, nf = ora.step_mixed(m, deg, U, 1e-5)
    after = ora.mixed_integrate(m, deg, U1)
    assert nf == 0
    assert np.all(np.abs(after - before) <= 1e-13 * np.abs(before).max())
    assert np.abs(U1 - U).max() > 1e-6


def test_mixed_rejects_bad_degrees(ora):
    m = _mesh(ora, SR, (2, 1, 1))
    with pytest.raises(ValueError):
        ora.rhs_mixed(m, np.array([0, 3], np.int32), np.zeros((5, 28)))


def test_mixed_ab3_equal_degrees_match_uniform(ora):
    """Adams-Bashforth 3 on a mixed-degree mesh whose degrees are all equal
    reproduces the uniform-degree steps bit for bit (its operator and its
    SSP-RK3 start both reduce to the uniform ones)."""
    m = _mesh(ora, SR, (3, 2, 2), 3)
    deg = np.full(12, 3, np.int32)
    U = _state(ora, SR, m, deg)
    # the random fields are steep on this coarse mesh (|L| ~ 1e5): a short step
    a, nfa = ora.evolve_ab3(m, U, 1e-6, 5)
    b, nfb = ora.evolve_ab3_mixed(m, deg, U, 1e-6, 5)
    assert nfa == nfb == 0
    assert np.array_equal(a, b)


@pytest.mark.parametrize("system", [NE, SR, MHD])
def test_mixed_ab3_conserves_totals(ora, system):
    m = _mesh(ora, system, (3, 2, 2))
    deg = synth.mixed_degrees(12, seed=1610)
    U = _state(ora, system, m, deg)
    before = ora.mixed_integrate(m, deg, U)
    U1, nf = ora.evolve_ab3_mixed(m, deg, U, 1e-6, 6)
    after = ora.mixed_integrate(m, deg, U1)
    assert nf == 0
    cons = slice(0, 8) if system == MHD else slice(0, 5)  # Phi is damped by kappa
    assert np.all(np.abs(after - before)[cons] <= 1e-13 * np.abs(before).max())
    assert np.abs(U1 - U).max() > 1e-3


def test_mixed_ab3_third_order_in_time(ora):
    """The advected SR wave on a checkerboard of degrees 3 and 4: against a
    reference of SSP-RK3 steps at dt/4, the AB3 error at dt and dt/2 falls
    by 2^3 (the spatial error is common to all three runs)."""
    g = 5.0 / 3.0
    K = 4
    m = ora.mesh(SR, (K, K, K), 2, g)
    e = np.arange(K ** 3)
    deg = np.where(((e % K) + (e // K) % K + e // (K * K)) % 2 == 0, 3, 4).astype(np.int32)
    xyz = ora.mixed_node_coords(m, deg)
    U0 = ora.prim2cons(SR, g, synth.smooth_flow(xyz, 0.0, 0.2, 2 * math.pi, (0.2, 0.2, 0.2)))
    # CFL ~ 0.05 at dt: measured ratios 1000, 18, 8 for dt = 0.008, 0.004,
    # 0.002 against half of each (the asymptotic range starts below 0.004)
    T, dt = 0.048, 0.002
    ref = U0
    for _ in range(192):
        ref, nf = ora.step_mixed(m, deg, ref, T / 192)
        assert nf == 0
    errs = []
    for h in (dt, dt / 2):
        U, nf = ora.evolve_ab3_mixed(m, deg, U0, h, int(round(T / h)))
        assert nf == 0
        errs.append(np.abs(U - ref).max())
    rate = math.log2(errs[0] / errs[1])
    assert 2.6 < rate < 3.6, (errs, rate)


def test_mixed_stable_dt(ora):
    """cfl h_min / lambda_max: equal degrees give the uniform value; on a
    checkerboard of degrees 2 and 5 with a constant state h_min is the
    degree-5 GLL gap (x_1 - x_0 = 1 - sqrt(1/3 + 2 sqrt(7) / 21)) times dx/2
    and lambda_max the constant state's speed."""
    g = 4.0 / 3.0
    m = _mesh(ora, SR, (3, 2, 2), 4)
    deg = np.full(12, 4, np.int32)
    U = _state(ora, SR, m, deg)
    assert ora.stable_dt_mixed(m, deg, U, 0.3) == ora.stable_dt(m, U, 0.3)
    deg = np.array([2, 5] * 6, np.int32)
    n = int(((deg + 1) ** 3).sum())
    prim = np.tile(np.array([[1.0], [0.3], [-0.2], [0.1], [0.5]]), (1, n))
    Uc = ora.prim2cons(SR, g, prim)
    mu = ora.mesh(SR, (1, 1, 1), 2, g)
    lam = ora.max_char_speed(mu, ora.prim2cons(SR, g, np.tile(prim[:, :1], (1, 27))))
    gap = 1.0 - math.sqrt(1.0 / 3.0 + 2.0 * math.sqrt(7.0) / 21.0)
    dxmin = min((np.array(m.hi[:]) - np.array(m.lo[:])) / np.array([3, 2, 2]))
    np.testing.assert_allclose(ora.stable_dt_mixed(m, deg, Uc, 0.3), 0.3 * 0.5 * dxmin * gap / lam, rtol=1e-14)


def _jump_mixed(ora, system, m, deg, seed=5):
    """x-only profile: smooth and monotone except for a drop across x = 0.37
    (so that no limiter decision rests on a rounding-level slope)."""
    xyz = ora.mixed_node_coords(m, deg)
    lo, hi = np.array(m.lo[:]), np.array(m.hi[:])
    x = (xyz[0] - lo[0]) / (hi[0] - lo[0])
    c = np.random.default_rng(seed).uniform(0.3, 1.0, size=4)
    step = x > 0.37
    one = np.ones_like(x)
    prim = np.stack([np.exp(c[0] * x) * np.where(step, 0.3, 1.0), 0.2 * np.exp(-c[1] * x), 0.1 * one,
                     0.05 * one, np.exp(c[3] * x) * np.where(step, 0.2, 1.0)])
    mag = None
    if system == MHD:
        mag = np.stack([one, 0.3 * np.exp(c[2] * x), 0.1 * one, 0.0 * one])
    return ora.prim2cons(system, m.gamma, prim, mag)


@pytest.mark.parametrize("system,N,lim", [(SR, 1, "minmod"), (NE, 3, "muscl"), (MHD, 2, "minmod")])
def test_mixed_limiter_equal_degrees_is_uniform(ora, system, N, lim):
    g = 4.0 / 3.0 if system else 1.4
    m = ora.mesh(system, (6, 2, 2), N, g, limiter=lim)
    deg = np.full(24, N, np.int32)
    U = _jump_mixed(ora, system, m, deg)
    a, na = ora.limit(m, U)
    b, nb, _ = ora.limit_mixed(m, deg, U)
    assert na == nb > 0
    assert np.array_equal(a, b)
    sa, _ = ora.step(m, U, 1e-4)
    sb, _ = ora.step_mixed(m, deg, U, 1e-4)
    assert np.array_equal(sa, sb)


@pytest.mark.parametrize("system", [NE, SR, MHD])
def test_mixed_limiter_invariants(ora, system):
    """On a random degree mix: element means (totals) unchanged; a constant
    state untouched; limited elements end up linear in their own nodes;
    elements far from the jump and the periodic wrap are left alone."""
    g = 4.0 / 3.0 if system else 1.4
    nel = (8, 2, 2)
    m = ora.mesh(system, nel, 2, g, limiter="minmod")
    deg = synth.mixed_degrees(32, seed=77, lo=1, hi=6)
    U = _jump_mixed(ora, system, m, deg)
    V, nlim, _ = ora.limit_mixed(m, deg, U)
    assert nlim > 0
    # totals (element means times volumes) are kept
    before, after = ora.mixed_integrate(m, deg, U), ora.mixed_integrate(m, deg, V)
    assert np.all(np.abs(after - before) <= 1e-13 * np.abs(before).max())
    # a constant state is never limited
    C = np.tile(U[:, :1], (1, U.shape[1]))
    W, nc, _ = ora.limit_mixed(m, deg, C)
    assert nc == 0 and np.array_equal(W, C)
    # changed components are linear along x (x-only data) in their element
    off = np.concatenate([[0], np.cumsum((deg + 1) ** 3)])
    xyz = ora.mixed_node_coords(m, deg)
    changed = []
    for e in range(32):
        sl = slice(off[e], off[e + 1])
        if np.array_equal(U[:, sl], V[:, sl]):
            continue
        changed.append(e % 8)
        x = xyz[0, sl]
        for v in range(U.shape[0]):
            if np.array_equal(U[v, sl], V[v, sl]):
                continue  # limiting acts per component
            fit = np.polyfit(x, V[v, sl], 1)
            assert np.abs(np.polyval(fit, x) - V[v, sl]).max() <= 1e-12 * max(1.0, np.abs(V[v, sl]).max())
    # x = 0.37 lies in element column 2; columns 0 and 7 meet at the wrap
    assert set(changed) <= {0, 1, 2, 3, 6, 7} and 2 in set(changed)


def test_mixed_step_with_limiter_conserves(ora):
    m = ora.mesh(SR, (8, 2, 2), 2, 4.0 / 3.0, limiter="muscl")
    deg = synth.mixed_degrees(32, seed=78, lo=1, hi=5)
    U = _jump_mixed(ora, SR, m, deg)
    before = ora.mixed_integrate(m, deg, U)
    V, nf = ora.step_mixed(m, deg, U, 2e-4)
    W, nf2 = ora.evolve_ab3_mixed(m, deg, U, 2e-4, 4)
    assert nf == nf2 == 0
    for X in (V, W):
        after = ora.mixed_integrate(m, deg, X)
        assert np.all(np.abs(after - before) <= 1e-12 * np.abs(before).max())
