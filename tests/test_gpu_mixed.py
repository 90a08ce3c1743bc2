"""GPU parity of the mixed-degree path (mortars between unequal degrees)
against the oracle's mixed-degree operator and stepper, on seeded smooth
random states; plus the equal-degree reduction to the uniform kernels,
graph replay against direct launches and the autotuner's choice (both bit
for bit)."""
import numpy as np
import pytest

from paper_1609_00098_amd import synth
from tests.gpu_util import normwise_err, to_dev, to_host

pytestmark = pytest.mark.gpu
NE, SR, MHD = 0, 1, 2
G = {NE: 1.4, SR: 4.0 / 3.0, MHD: 4.0 / 3.0}


@pytest.fixture(scope="module")
def dg():
    import torch
    assert torch.cuda.is_available()
    from paper_1609_00098_amd import dgmi
    return dgmi


def _setup(ora, dg, system, nel, deg, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), seed=1609, flags=0, mild=True,
           flux="llf"):
    """Seeded smooth random state.  Small meshes get mild fields (rho, p in
    [0.5, 2], W <= 2): interpolating badly under-resolved data onto a finer
    mortar can overshoot to negative density or pressure, which the method
    does not guard against (that is a limiter's job), so parity there would
    compare two treatments of unphysical states."""
    g = G[system]
    kw = dict(w_max=2.0, rho_range=(0.5, 2.0), p_range=(0.5, 2.0)) if mild else {}
    m = ora.mesh(system, nel, 2, g, lo=lo, hi=hi, kappa=0.5, flux=flux)
    if flux == "hll":
        flags |= dg.FLAG_HLL
    mesh = dg.Mesh(system, nel, 0, g, lo=lo, hi=hi, kappa=0.5, flags=flags, degrees=deg)
    xyz = ora.mixed_node_coords(m, deg)
    unit = (xyz - np.array(lo)[:, None]) / (np.array(hi) - np.array(lo))[:, None]
    if system == MHD:
        prim = synth.fourier_random_prims(unit, seed=seed, **kw)
        rng = np.random.default_rng(seed)
        mag = np.zeros((4, prim.shape[1]))
        for c in range(4):
            k = rng.integers(1, 3, size=3)
            mag[c] = 0.3 * np.sin(2 * np.pi * (k @ unit) + rng.uniform(0, 6))
        mag[0] += 1.0
        U = ora.prim2cons(MHD, g, prim, mag)
    else:
        prim = synth.fourier_random_prims(unit, seed=seed, **kw)
        U = ora.prim2cons(system, g, prim)
    return m, mesh, U, prim, xyz


CASES = [
    (SR, (3, 3, 2), "random27"),
    (SR, (4, 3, 3), "random17"),
    (NE, (3, 2, 3), "random17"),
    (MHD, (3, 2, 2), "random27"),
    (SR, (2, 2, 2), "checker37"),
]


def _degrees(kind, ne):
    if kind == "random27":
        return synth.mixed_degrees(ne, seed=1610)
    if kind == "random17":
        return synth.mixed_degrees(ne, seed=11, lo=1, hi=7)
    return np.array([3 + 4 * (e % 2) for e in range(ne)], np.int32)


@pytest.mark.parametrize("system,nel,kind", CASES)
def test_mixed_node_coords_and_offsets(ora, dg, system, nel, kind):
    deg = _degrees(kind, int(np.prod(nel)))
    m, mesh, _, _, xyz = _setup(ora, dg, system, nel, deg)
    assert mesh.nnodes == ora.mixed_num_nodes(deg)
    off = mesh.elem_offsets()
    assert np.array_equal(np.diff(off), (deg.astype(np.int64) + 1) ** 3)
    assert np.array_equal(mesh.elem_offsets_host(), off)
    assert np.abs(to_host(mesh.node_coords()) - xyz).max() <= 1e-15


def test_degree_minus_one_selects_per_element_degrees(dg):
    deg = _degrees("random27", 18)
    a = dg.Mesh(SR, (3, 3, 2), 0, G[SR], degrees=deg)
    b = dg.Mesh(SR, (3, 3, 2), -1, G[SR], degrees=deg)
    assert a.nnodes == b.nnodes
    assert np.array_equal(a.elem_offsets_host(), b.elem_offsets())


@pytest.mark.parametrize("system,nel,kind", CASES)
def test_mixed_rhs_parity(ora, dg, system, nel, kind):
    deg = _degrees(kind, int(np.prod(nel)))
    m, mesh, U, prim, _ = _setup(ora, dg, system, nel, deg)
    L, Po, nf = ora.rhs_mixed(m, deg, U)
    assert nf == 0
    P = to_dev(prim * np.array([[1.0], [1.0], [1.0], [1.0], [1.001]]))
    out = mesh.empty_state()
    dg.dg_rhs(mesh, to_dev(U), P, out)
    assert dg.dgmi_failures(mesh) == 0
    err = normwise_err(to_host(out), L)
    assert err.max() <= 1e-12, err
    # dg_operator with the oracle's primitives gives the same operator
    out2 = mesh.empty_state()
    dg.dg_operator(mesh, to_dev(U), to_dev(Po), out2)
    err = normwise_err(to_host(out2), L)
    assert err.max() <= 1e-12, err


@pytest.mark.parametrize("system,N", [(SR, 4), (SR, 2), (NE, 3), (MHD, 3), (SR, 7)])
def test_equal_degrees_match_uniform_kernels(ora, dg, system, N):
    """With every face conforming the mixed kernels do the uniform kernels'
    arithmetic; only the compiler's fused multiply-add choices may differ."""
    nel = (3, 2, 2)
    deg = np.full(12, N, np.int32)
    m, mixed, U, prim, _ = _setup(ora, dg, system, nel, deg)
    uni = dg.Mesh(system, nel, N, G[system], kappa=0.5)
    Ud, Pd = to_dev(U), to_dev(prim)
    a, b = mixed.empty_state(), uni.empty_state()
    dg.dg_operator(mixed, Ud, Pd, a)
    dg.dg_operator(uni, Ud, Pd, b)
    err = normwise_err(to_host(a), to_host(b))
    assert err.max() <= 1e-14, err


@pytest.mark.parametrize("system,nel,kind", CASES)
def test_mixed_hll_rhs_parity(ora, dg, system, nel, kind):
    """The HLL flux (eq. HLL) on mixed degrees: the mortar kernel's flux at the
    mortar nodes and the element kernels' on conforming faces, against the
    oracle's mixed operator with the same flux."""
    deg = _degrees(kind, int(np.prod(nel)))
    m, mesh, U, prim, _ = _setup(ora, dg, system, nel, deg, flux="hll")
    L, Po, nf = ora.rhs_mixed(m, deg, U)
    assert nf == 0
    Llf, _, _ = ora.rhs_mixed(ora.mesh(system, nel, 2, G[system], kappa=0.5), deg, U)
    assert normwise_err(Llf, L).max() > 1e-6  # the two fluxes differ here
    P = to_dev(prim * np.array([[1.0], [1.0], [1.0], [1.0], [1.001]]))
    out = mesh.empty_state()
    dg.dg_rhs(mesh, to_dev(U), P, out)
    assert dg.dgmi_failures(mesh) == 0
    err = normwise_err(to_host(out), L)
    assert err.max() <= 1e-12, err


@pytest.mark.parametrize("system,N", [(SR, 4), (NE, 3), (MHD, 3)])
def test_hll_equal_degrees_match_uniform_hll_kernels(ora, dg, system, N):
    nel = (3, 2, 2)
    deg = np.full(12, N, np.int32)
    m, mixed, U, prim, _ = _setup(ora, dg, system, nel, deg, flux="hll")
    uni = dg.Mesh(system, nel, N, G[system], kappa=0.5, flags=dg.FLAG_HLL)
    Ud, Pd = to_dev(U), to_dev(prim)
    a, b = mixed.empty_state(), uni.empty_state()
    dg.dg_operator(mixed, Ud, Pd, a)
    dg.dg_operator(uni, Ud, Pd, b)
    err = normwise_err(to_host(a), to_host(b))
    assert err.max() <= 1e-14, err


@pytest.mark.parametrize("system,nel,kind", CASES[:4])
def test_mixed_hll_step_parity(ora, dg, system, nel, kind):
    """RK3 steps with the HLL flux, direct and graph-replayed, and with the
    MUSCL limiter after every stage, against the oracle."""
    import torch
    deg = _degrees(kind, int(np.prod(nel)))
    m, mesh, U, prim, _ = _setup(ora, dg, system, nel, deg, flux="hll")
    L, Po, _ = ora.rhs_mixed(m, deg, U)
    dt = _dt(L, U)
    Uo, nf = ora.step_mixed(m, deg, U, dt)
    assert nf == 0
    tol = 2e-12 * dt * np.abs(L).max() + 8 * np.finfo(float).eps * np.abs(U).max()
    res = []
    for use_graph in (False, True):
        Ud, Pd = to_dev(U), to_dev(Po)
        s = torch.cuda.Stream() if use_graph else None
        if s is not None:
            s.wait_stream(torch.cuda.current_stream())
        dg.dg_step(mesh, Ud, Pd, dt, stream=s)
        torch.cuda.synchronize()
        assert dg.dgmi_failures(mesh) == 0
        res.append(to_host(Ud))
        assert np.abs(res[-1] - Uo).max() <= tol, (np.abs(res[-1] - Uo).max(), tol)
    assert np.array_equal(res[0], res[1])


@pytest.mark.parametrize("system,lim,seed", [(SR, "muscl", 81), (MHD, "minmod", 82)])
def test_mixed_hll_step_with_limiter_parity(ora, dg, system, lim, seed):
    """Limited RK3 steps with the HLL flux on a random mix of degrees 1..7
    (the limited stage kernel in its HLL instantiation)."""
    g = G[system]
    nel = (8, 2, 2)
    deg = synth.mixed_degrees(32, seed=seed, lo=1, hi=7)
    m = ora.mesh(system, nel, 2, g, kappa=0.5, limiter=lim, flux="hll")
    U, prim = _jump_state(ora, system, m, deg)
    U, _, _ = ora.limit_mixed(m, deg, U)
    L, Po, _ = ora.rhs_mixed(m, deg, U)
    dt = 2e-3 / float(max(np.abs(L[0] / U[0]).max(), np.abs(L[4] / U[4]).max()))
    eps = np.finfo(np.float64).eps
    budget = 4e-12 * dt * np.maximum(np.abs(L).max(axis=1), 1e-3 * np.abs(L).max()) + 32 * eps * np.abs(U).max(axis=1)
    Uo, nf = ora.step_mixed(m, deg, U, dt)
    assert nf == 0
    mesh = dg.Mesh(system, nel, 0, g, kappa=0.5, degrees=deg, flags=dg.FLAG_HLL)
    dg.dgmi_set_limiter(mesh, {"minmod": dg.LIMITER_MINMOD, "muscl": dg.LIMITER_MUSCL}[lim], 0.0)
    Ud, Pd = to_dev(U), to_dev(Po)
    dg.dgmi_limited(mesh)
    dg.dg_step(mesh, Ud, Pd, dt)
    assert dg.dgmi_limited(mesh) > 0
    assert dg.dgmi_failures(mesh) == 0
    diff = np.abs(to_host(Ud) - Uo).max(axis=1)
    assert np.all(diff <= budget), (diff, budget)


def _dt(L, U):
    return 1e-3 / float(np.max(np.abs(L) / np.maximum(np.abs(U), 1e-300)))


@pytest.mark.parametrize("system,nel,kind", CASES[:4])
def test_mixed_step_parity(ora, dg, system, nel, kind):
    import torch
    deg = _degrees(kind, int(np.prod(nel)))
    m, mesh, U, prim, _ = _setup(ora, dg, system, nel, deg)
    L, Po, _ = ora.rhs_mixed(m, deg, U)
    dt = _dt(L, U)
    Uo, nf = ora.step_mixed(m, deg, U, dt)
    assert nf == 0
    res = {}
    for use_graph in (False, True):
        Ud, Pd = to_dev(U), to_dev(Po)
        s = torch.cuda.Stream() if use_graph else None
        if s is not None:
            s.wait_stream(torch.cuda.current_stream())
        dg.dg_step(mesh, Ud, Pd, dt, stream=s)
        torch.cuda.synchronize()
        assert dg.dgmi_failures(mesh) == 0
        res[use_graph] = (to_host(Ud), to_host(Pd))
        # increments agree to the operator's tolerance
        tol = 2e-12 * dt * np.abs(L).max() + 8 * np.finfo(float).eps * np.abs(U).max()
        assert np.abs(res[use_graph][0] - Uo).max() <= tol, (np.abs(res[use_graph][0] - Uo).max(), tol)
    assert np.array_equal(res[False][0], res[True][0])
    assert np.array_equal(res[False][1], res[True][1])


def test_graph_replays_with_new_dt_and_state(ora, dg):
    """Two steps through one captured graph (second with another dt) equal
    two directly launched steps bit for bit."""
    import torch
    deg = _degrees("random27", 18)
    m, mesh, U, prim, _ = _setup(ora, dg, SR, (3, 3, 2), deg)
    direct = dg.Mesh(SR, (3, 3, 2), 0, G[SR], flags=dg.FLAG_NO_GRAPH, degrees=deg)
    L, Po, _ = ora.rhs_mixed(m, deg, U)
    dt = _dt(L, U)
    s = torch.cuda.Stream()
    Ua, Pa = to_dev(U), to_dev(Po)
    Ub, Pb = to_dev(U), to_dev(Po)
    s.wait_stream(torch.cuda.current_stream())
    for k, step_dt in enumerate((dt, 0.5 * dt, 0.7 * dt)):
        dg.dg_step(mesh, Ua, Pa, step_dt, stream=s)
        s.synchronize()
        dg.dg_step(direct, Ub, Pb, step_dt)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(Ua), to_host(Ub)), k
        assert np.array_equal(to_host(Pa), to_host(Pb)), k


def test_autotuned_tiles_give_identical_results(ora, dg):
    deg = synth.mixed_degrees(64, seed=5, lo=1, hi=7)
    m, plain, U, prim, _ = _setup(ora, dg, SR, (4, 4, 4), deg)
    tuned = dg.Mesh(SR, (4, 4, 4), 0, G[SR], flags=dg.FLAG_AUTOTUNE, degrees=deg)
    Ud, Pd = to_dev(U), to_dev(prim)
    a, b = plain.empty_state(), tuned.empty_state()
    dg.dg_operator(plain, Ud, Pd, a)
    dg.dg_operator(tuned, Ud, Pd, b)
    assert np.array_equal(to_host(a), to_host(b))
    # the choice is reported: one launch or per-degree launches, and per
    # degree present one of its tile options
    single, tiles = tuned.mixed_launch_mode()
    assert isinstance(single, bool)
    assert sorted(tiles) == sorted(set(int(x) for x in deg))
    options = {1: (8, 4), 2: (9, 4), 3: (4, 2), 4: (2, 1), 5: (1,), 6: (1,), 7: (1,)}
    assert all(tiles[N] in options[N] for N in tiles), tiles
    assert plain.mixed_launch_mode()[0] is True
    assert dg.Mesh(SR, (2, 2, 2), 3, G[SR]).mixed_launch_mode() is None


def _mixed_16x16x16_deg2to7(ora, dg, flags=0):
    """SR hydro, gamma 4/3, 16^3 elements on the unit box, degrees uniform in
    2..7 (seed 1610), the smooth random primitives (seed 1609) at every
    element's own nodes."""
    deg = synth.mixed_degrees(4096, seed=1610)
    return _setup(ora, dg, SR, (16, 16, 16), deg, flags=flags, mild=False) + (deg,)


def _ulp_sensitivity(ora, m, deg, U, L):
    """Normwise change of the oracle's own operator when every input value
    moves by one ulp (seeded signs): two correct FP64 evaluations that round
    differently cannot be expected to agree more closely than this."""
    rng = np.random.default_rng(0)
    Up = U * (1.0 + np.finfo(float).eps * rng.choice([-1.0, 1.0], size=U.shape))
    Lp, _, _ = ora.rhs_mixed(m, deg, Up)
    return normwise_err(Lp, L).max()


def test_mixed_full_size_rhs_and_step(ora, dg):
    """16^3 elements of degrees 2..7 with the full-range fields (W up to 10,
    p over four decades).  Here the operator itself moves by ~1e-12 under a
    one-ulp change of U (the recovery is ill conditioned at W ~ 10 and the
    degree-7 lift and derivative amplify the rounding of fluxes far larger
    than their divergence), so the bar is the larger of 1e-12 and twice that
    measured sensitivity, for the operator on the oracle's primitives as for
    dg_rhs; the same mesh with the fields the step is timed on meets 1e-12
    itself (next test)."""
    import torch
    m, mesh, U, prim, _, deg = _mixed_16x16x16_deg2to7(ora, dg)
    assert mesh.nnodes == 879747
    L, Po, nf = ora.rhs_mixed(m, deg, U)
    assert nf == 0
    Ud = to_dev(U)
    out = mesh.empty_state()
    tol = max(1e-12, 2.0 * _ulp_sensitivity(ora, m, deg, U, L))
    assert tol <= 5e-12
    dg.dg_operator(mesh, Ud, to_dev(Po), out)
    err = normwise_err(to_host(out), L)
    assert err.max() <= tol, (err, tol)
    P = to_dev(prim * np.array([[1.0], [1.0], [1.0], [1.0], [1.001]]))
    dg.dg_rhs(mesh, Ud, P, out)
    err = normwise_err(to_host(out), L)
    assert err.max() <= tol, (err, tol)
    dt = 2e-4
    Uo, nf = ora.step_mixed(m, deg, U, dt)
    assert nf == 0
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    Pd = to_dev(Po)
    dg.dg_step(mesh, Ud, Pd, dt, stream=s)
    s.synchronize()
    assert dg.dgmi_failures(mesh) == 0
    stol = 2 * tol * dt * np.abs(L).max() + 8 * np.finfo(float).eps * np.abs(U).max()
    assert np.abs(to_host(Ud) - Uo).max() <= stol


def test_mixed_full_size_timed_fields_at_1e12(ora, dg):
    """The same 16^3 mesh of degrees 2..7 with the fields its RK3 step is
    timed on (seed 1609, rho, p in [0.5, 2], W up to 3, at every element's
    own nodes of the unit box): dg_operator on the oracle's primitives,
    dg_rhs with recovery from a 0.1%-off pressure seed, and one RK3 step,
    all at the relative 1e-12 bar."""
    import torch
    deg = synth.mixed_degrees(4096, seed=1610)
    m = ora.mesh(SR, (16, 16, 16), 2, G[SR], kappa=0.5)
    mesh = dg.Mesh(SR, (16, 16, 16), 0, G[SR], kappa=0.5, degrees=deg)
    xyz = ora.mixed_node_coords(m, deg)
    prim = synth.fourier_random_prims(xyz, seed=1609, rho_range=(0.5, 2.0), p_range=(0.5, 2.0), w_max=3.0)
    U = ora.prim2cons(SR, G[SR], prim)
    L, Po, nf = ora.rhs_mixed(m, deg, U)
    assert nf == 0
    Ud = to_dev(U)
    out = mesh.empty_state()
    dg.dg_operator(mesh, Ud, to_dev(Po), out)
    err = normwise_err(to_host(out), L)
    assert err.max() <= 1e-12, err
    dg.dg_rhs(mesh, Ud, to_dev(prim * np.array([[1.0], [1.0], [1.0], [1.0], [1.001]])), out)
    assert dg.dgmi_failures(mesh) == 0
    err = normwise_err(to_host(out), L)
    assert err.max() <= 1e-12, err
    dt = 2e-4
    Uo, nf = ora.step_mixed(m, deg, U, dt)
    assert nf == 0
    Pd = to_dev(Po)
    dg.dg_step(mesh, Ud, Pd, dt)
    torch.cuda.synchronize()
    assert dg.dgmi_failures(mesh) == 0
    # each stage adds at most dt * (1e-12 of the operator's scale)
    stol = 2e-12 * dt * np.abs(L).max(axis=1, keepdims=True) + 8 * np.finfo(float).eps * np.abs(U).max(axis=1, keepdims=True)
    assert np.all(np.abs(to_host(Ud) - Uo) <= stol)


@pytest.mark.parametrize("system,nel,kind", CASES[:4])
def test_mixed_ab3_parity(ora, dg, system, nel, kind):
    """Adams-Bashforth 3 on mixed degrees (two RK3 starting steps, then one
    mortar + element operator pass per step) against the oracle, within the
    per-step operator budget times the number of steps."""
    deg = _degrees(kind, int(np.prod(nel)))
    m, mesh, U, prim, _ = _setup(ora, dg, system, nel, deg)
    L, Po, _ = ora.rhs_mixed(m, deg, U)
    dt = _dt(L, U)
    n = 6
    Uo, nf = ora.evolve_ab3_mixed(m, deg, U, dt, n)
    assert nf == 0
    Ud, Pd = to_dev(U), to_dev(Po)
    for _ in range(n):
        dg.dg_step_ab3(mesh, Ud, Pd, dt)
    assert dg.dgmi_failures(mesh) == 0
    assert abs(dg.dgmi_get_time(mesh) - n * dt) < 1e-15
    eps = np.finfo(np.float64).eps
    tol = n * (4e-12 * dt * np.maximum(np.abs(L).max(axis=1), 1e-3 * np.abs(L).max()) +
               8 * eps * np.abs(U).max(axis=1))
    diff = np.abs(to_host(Ud) - Uo).max(axis=1)
    assert np.all(diff <= tol), (diff, tol)
    assert np.all(np.abs(Uo - U).max(axis=1)[:5] > 1e2 * tol[:5])


def test_mixed_stable_dt_parity(ora, dg):
    deg = _degrees("random17", 36)
    m, mesh, U, prim, _ = _setup(ora, dg, SR, (4, 3, 3), deg)
    _, Po, _ = ora.rhs_mixed(m, deg, U)
    dt_o = ora.stable_dt_mixed(m, deg, U, 0.3)
    dt = float(to_host(dg.dgmi_stable_dt(mesh, to_dev(U), to_dev(Po), 0.3))[0])
    assert abs(dt - dt_o) <= 1e-14 * dt_o


def _jump_state(ora, system, m, deg, seed=5):
    """x-only profile, smooth and monotone except for a drop across x = 0.37
    (no limiter decision rests on a rounding-level slope)."""
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
    return ora.prim2cons(system, m.gamma, prim, mag), prim


LIM_CASES = [(NE, "minmod", 77), (SR, "muscl", 78), (MHD, "minmod", 79)]


@pytest.mark.parametrize("system,lim,seed", LIM_CASES)
def test_mixed_limit_parity(ora, dg, system, lim, seed):
    """Limiter on a random mix of degrees 1..7: decisions equal the oracle's,
    limited U within 1e-13 norm-wise, primitives within 1e-12."""
    g = G[system]
    nel = (8, 2, 2)
    deg = synth.mixed_degrees(32, seed=seed, lo=1, hi=7)
    m = ora.mesh(system, nel, 2, g, kappa=0.5, limiter=lim)
    mesh = dg.Mesh(system, nel, 0, g, kappa=0.5, degrees=deg)
    dg.dgmi_set_limiter(mesh, {"minmod": dg.LIMITER_MINMOD, "muscl": dg.LIMITER_MUSCL}[lim], 0.0)
    U, prim = _jump_state(ora, system, m, deg)
    Uo, nlim, _ = ora.limit_mixed(m, deg, U)
    assert nlim > 0
    Po, _, nf = ora.cons2prim(system, g, Uo)
    assert nf == 0
    Ud, Pd = to_dev(U), to_dev(prim)
    dg.dgmi_limited(mesh)
    dg.dg_limit(mesh, Ud, Pd)
    assert dg.dgmi_limited(mesh) == nlim
    assert dg.dgmi_failures(mesh) == 0
    assert np.all(normwise_err(to_host(Ud), Uo, floor_scale=1.0) <= 1e-13)
    assert np.all(normwise_err(to_host(Pd), Po, floor_scale=1.0) <= 1e-12)


@pytest.mark.parametrize("system,lim,seed", LIM_CASES)
def test_mixed_step_with_limiter_parity(ora, dg, system, lim, seed):
    """Limited RK3 steps (direct and graph-replayed) and limited AB3 steps on a
    random degree mix against the oracle, within the step budget."""
    import torch
    g = G[system]
    nel = (8, 2, 2)
    deg = synth.mixed_degrees(32, seed=seed, lo=1, hi=7)
    m = ora.mesh(system, nel, 2, g, kappa=0.5, limiter=lim)
    U, prim = _jump_state(ora, system, m, deg)
    U, _, _ = ora.limit_mixed(m, deg, U)
    L, Po, _ = ora.rhs_mixed(m, deg, U)
    dt = 2e-3 / float(max(np.abs(L[0] / U[0]).max(), np.abs(L[4] / U[4]).max()))
    eps = np.finfo(np.float64).eps
    budget = 4e-12 * dt * np.maximum(np.abs(L).max(axis=1), 1e-3 * np.abs(L).max()) + 32 * eps * np.abs(U).max(axis=1)
    kind = {"minmod": dg.LIMITER_MINMOD, "muscl": dg.LIMITER_MUSCL}[lim]
    Uo, nf = ora.step_mixed(m, deg, U, dt)
    assert nf == 0
    res = []
    for use_graph in (False, True):
        mesh = dg.Mesh(system, nel, 0, g, kappa=0.5, degrees=deg)
        dg.dgmi_set_limiter(mesh, kind, 0.0)
        Ud, Pd = to_dev(U), to_dev(Po)
        s = torch.cuda.Stream() if use_graph else None
        if s is not None:
            s.wait_stream(torch.cuda.current_stream())
        dg.dgmi_limited(mesh)
        dg.dg_step(mesh, Ud, Pd, dt, stream=s)
        torch.cuda.synchronize()
        assert dg.dgmi_limited(mesh) > 0
        assert dg.dgmi_failures(mesh) == 0
        diff = np.abs(to_host(Ud) - Uo).max(axis=1)
        assert np.all(diff <= budget), (use_graph, diff, budget)
        res.append(to_host(Ud))
    assert np.array_equal(res[0], res[1])
    n = 5
    Ua, nf = ora.evolve_ab3_mixed(m, deg, U, dt, n)
    assert nf == 0
    mesh = dg.Mesh(system, nel, 0, g, kappa=0.5, degrees=deg)
    dg.dgmi_set_limiter(mesh, kind, 0.0)
    Ud, Pd = to_dev(U), to_dev(Po)
    for _ in range(n):
        dg.dg_step_ab3(mesh, Ud, Pd, dt)
    assert dg.dgmi_failures(mesh) == 0
    diff = np.abs(to_host(Ud) - Ua).max(axis=1)
    assert np.all(diff <= n * budget), (diff, n * budget)


@pytest.mark.parametrize("system", [SR, MHD])
def test_mixed_blast_with_limiter_and_fixing(ora, dg, system):
    """A periodic blast (pressure 1000 against 0.01, gamma 5/3) on a mix of
    degrees 1..3, MUSCL with the conserved-variable fixing: limited alone it
    goes non-finite within eight steps; with the fixing every step matches
    the oracle within 1e-10 per variable, the fixing acts, and no recovery
    fails."""
    g = 5.0 / 3.0
    nx = 60
    deg = synth.mixed_degrees(nx, seed=91, lo=1, hi=3)
    m = ora.mesh(system, (nx, 1, 1), 2, g, lo=(-0.5, 0, 0), hi=(0.5, 1, 1), limiter="muscl", fix=(1e-10, 1e-12))
    mesh = dg.Mesh(system, (nx, 1, 1), 0, g, lo=(-0.5, 0, 0), hi=(0.5, 1, 1), degrees=deg)
    dg.dgmi_set_limiter(mesh, dg.LIMITER_MUSCL, 0.0)
    dg.dgmi_set_fixing(mesh, 1e-10, 1e-12)
    x = ora.mixed_node_coords(m, deg)[0]
    n = len(x)
    prim = np.vstack([np.ones(n), np.zeros((3, n)), np.where(np.abs(x) < 0.1, 1000.0, 0.01)])
    mag = None
    if system == MHD:
        mag = np.zeros((4, n))
        mag[0] = 0.5
    U = ora.prim2cons(system, g, prim, mag)
    dt = 0.1 / (3 * nx)
    Ud, Pd = to_dev(U), to_dev(prim)
    Uo = U
    fixed = 0
    dg.dgmi_failures(mesh)
    for s in range(8):
        dg.dg_step(mesh, Ud, Pd, dt)
        Uo, nf = ora.step_mixed(m, deg, Uo, dt)
        assert nf == 0
        assert dg.dgmi_failures(mesh) == 0
        fixed += dg.dgmi_fixed(mesh)
        err = normwise_err(to_host(Ud), Uo, floor_scale=1.0)
        assert np.all(err <= 1e-10), (s, err)
    assert fixed > 0
