"""Pins of the oracle's pointwise physics against independent mathematics.

* conserved variables and fluxes of the relativistic systems against the
  stress-energy tensor T^{mu nu} built from 4-vectors (textbook route, not the
  3+1 formulas the oracle uses);
* largest wave speeds against eigenvalues of a finite-difference flux
  Jacobian (the characteristic decomposition section);
* recovery: round trips, exact limits, uniqueness of the root by brute-force
  scan, backward residual, failure detection.
"""
import numpy as np
import pytest

from paper_1609_00098_amd import synth

NE, SR, MHD = 0, 1, 2


def _stress_energy(rho, v, p, B, gamma):
    """Flat-space ideal-MHD T^{mu nu} = (rho h + b^2) u u + (p + b^2/2) eta - b b."""
    W = 1.0 / np.sqrt(1.0 - v @ v)
    h = 1.0 + gamma * p / ((gamma - 1.0) * rho)
    u = W * np.array([1.0, *v])
    b0 = W * (B @ v)
    b = np.array([b0, *(B / W + b0 * v)])
    eta = np.diag([-1.0, 1.0, 1.0, 1.0])
    b2 = -b[0] ** 2 + b[1:] @ b[1:]
    T = (rho * h + b2) * np.outer(u, u) + (p + 0.5 * b2) * eta - np.outer(b, b)
    return T, rho * W, W


@pytest.mark.parametrize("system", [SR, MHD])
def test_relativistic_cons_and_flux_from_stress_energy(ora, system):
    g = 4.0 / 3.0
    prim, mag = synth.srmhd_samples(200, seed=7, w_max=5.0)
    if system == SR:
        mag[:] = 0.0
    U = ora.prim2cons(system, g, prim, mag)
    for q in range(0, 200, 7):
        rho, v, p, B = prim[0, q], prim[1:4, q], prim[4, q], mag[:3, q]
        T, D, W = _stress_energy(rho, v, p, B, g)
        assert abs(U[0, q] - D) <= 1e-13 * D
        scale = T[0, 0]
        assert np.abs(U[1:4, q] - T[0, 1:]).max() <= 1e-12 * scale
        assert abs(U[4, q] - (T[0, 0] - D)) <= 1e-12 * scale
        for d in range(3):
            F = ora.flux(system, g, d, U[:, q:q + 1], prim[:, q:q + 1])[:, 0]
            assert abs(F[0] - D * v[d]) <= 1e-13 * D
            assert np.abs(F[1:4] - T[1 + d, 1:]).max() <= 1e-12 * scale
            assert abs(F[4] - (T[0, 1 + d] - D * v[d])) <= 1e-12 * scale
            if system == MHD:
                # induction: F^d(B^i) = v^d B^i - v^i B^d + delta Phi, F^d(Phi) = B^d
                Fi = v[d] * B - v * B[d]
                Fi[d] += U[8, q]
                assert np.abs(F[5:8] - Fi).max() <= 1e-13 * (1 + np.abs(B).max())
                assert F[8] == B[d]


def _fd_jacobian(ora, system, g, d, u):
    n = len(u)
    J = np.zeros((n, n))

    def F(uu):
        prim, fail, _ = ora.cons2prim(system, g, uu[:, None])
        assert not fail.any()
        return ora.flux(system, g, d, uu[:, None], prim)[:, 0]

    for c in range(n):
        h = 1e-6 * max(abs(u[c]), 1e-3)
        up, um = u.copy(), u.copy()
        up[c] += h
        um[c] -= h
        J[:, c] = (F(up) - F(um)) / (2 * h)
    return J


@pytest.mark.parametrize("system", [NE, SR])
def test_max_speed_equals_jacobian_spectral_radius(ora, system):
    g = 5.0 / 3.0
    rng = np.random.default_rng(3)
    for q in range(6):
        if system == NE:
            prim = np.array([[rng.uniform(0.5, 2)], [rng.uniform(-1, 1)], [rng.uniform(-1, 1)],
                             [rng.uniform(-1, 1)], [rng.uniform(0.5, 2)]])
        else:
            prim = synth.sr_samples(1, seed=100 + q, w_max=4.0)
        U = ora.prim2cons(system, g, prim)
        for d in range(3):
            J = _fd_jacobian(ora, system, g, d, U[:, 0])
            lam = np.abs(np.linalg.eigvals(J)).max()
            a = ora.max_speed(system, g, d, U, prim)[0, 0]
            assert abs(a - lam) < 1e-5 * max(1.0, lam)


def test_mhd_speed_bounds_jacobian_and_cleaning_split(ora):
    """The fast-speed bound dominates every eigenvalue of the 7-variable
    sub-system, and the (B_n, Phi) sub-system has speeds exactly +-1."""
    g = 4.0 / 3.0
    prim, mag = synth.srmhd_samples(6, seed=11, w_max=3.0, sigma_range=(1e-2, 3.0), p_over_rho=(1e-2, 1e1))
    U = ora.prim2cons(MHD, g, prim, mag)
    for q in range(6):
        for d in range(3):
            J = _fd_jacobian(ora, MHD, g, d, U[:, q])
            a = ora.max_speed(MHD, g, d, U[:, q:q + 1], prim[:, q:q + 1])[:, 0]
            sub = [5 + d, 8]
            rest = [c for c in range(9) if c not in sub]
            Jc = J[np.ix_(sub, sub)]
            assert np.allclose(np.sort(np.linalg.eigvals(Jc).real), [-1.0, 1.0], atol=1e-6)
            assert a[5 + d] == 1.0 and a[8] == 1.0
            # the (B_n, Phi) fluxes do not depend on the other variables
            assert np.abs(J[np.ix_(sub, rest)]).max() < 1e-6
            lam = np.abs(np.linalg.eigvals(J[np.ix_(rest, rest)])).max()
            assert lam <= a[0] * (1 + 1e-5) + 1e-8
            assert a[0] < 1.0


def _perpendicular_field_states(d, rng, n):
    """SRMHD primitives with the velocity along e_d (zero for the first two)
    and the field across it: magnetisation sigma = b^2/rho in [1e-2, 10],
    p/rho in [1e-2, 10], |v| up to 0.9."""
    prim = np.zeros((5, n))
    mag = np.zeros((4, n))
    for q in range(n):
        rho = 10 ** rng.uniform(-1, 1)
        p = rho * 10 ** rng.uniform(-2, 1)
        vn = 0.0 if q < 2 else rng.uniform(-0.9, 0.9)
        W = 1.0 / np.sqrt(1.0 - vn * vn)
        sigma = 10 ** rng.uniform(-2, 1)
        th = rng.uniform(0, 2 * np.pi)
        t1, t2 = [k for k in range(3) if k != d]
        Bhat = np.zeros(3)
        Bhat[t1], Bhat[t2] = np.cos(th), np.sin(th)
        # B.v = 0, so b^2 = B^2 / W^2
        prim[:, q] = [rho, 0, 0, 0, p]
        prim[1 + d, q] = vn
        mag[:3, q] = W * np.sqrt(sigma * rho) * Bhat
    return prim, mag


@pytest.mark.parametrize("d", [0, 1, 2])
def test_mhd_fast_speed_exact_for_field_across_the_normal(ora, d):
    """With B perpendicular to e_d and v along e_d (or zero) the fast
    magnetosonic wave crosses the field at a right angle in the fluid frame,
    where its speed is exactly c_f^2 = v_A^2 + c_s^2 (1 - v_A^2) with
    v_A^2 = b^2/(rho h + b^2), and the collinear boost makes the lab-frame
    speeds (v_n +- c_f)/(1 +- v_n c_f).  So the fluid part's largest speed and
    both signed bounds must equal the extreme eigenvalues of the
    finite-difference Jacobian of the 7-variable sub-system exactly (to the
    difference quotient's accuracy), which fails for a slip such as
    v_A^2 = b^2/(rho h) or a fast speed without the (1 - v_A^2) factor."""
    g = 4.0 / 3.0
    rng = np.random.default_rng(40 + d)
    prim, mag = _perpendicular_field_states(d, rng, 8)
    U = ora.prim2cons(MHD, g, prim, mag)
    a = ora.max_speed(MHD, g, d, U, prim)
    lm, lp = ora.wave_speeds(MHD, g, d, U, prim)
    sub = [5 + d, 8]
    rest = [c for c in range(9) if c not in sub]
    for q in range(U.shape[1]):
        J = _fd_jacobian(ora, MHD, g, d, U[:, q])
        ev = np.linalg.eigvals(J[np.ix_(rest, rest)])
        assert np.abs(ev.imag).max() < 1e-6
        ev = ev.real
        for c in rest:
            assert abs(a[c, q] - np.abs(ev).max()) <= 1e-6, (q, c, a[c, q], ev)
            assert abs(lp[c, q] - ev.max()) <= 1e-6 and abs(lm[c, q] - ev.min()) <= 1e-6, (q, c, ev)
        # the cleaning pair moves at the light speed
        assert a[5 + d, q] == 1.0 and a[8, q] == 1.0
        assert lm[5 + d, q] == -1.0 and lp[5 + d, q] == 1.0 and lm[8, q] == -1.0 and lp[8, q] == 1.0


@pytest.mark.parametrize("system", [NE, SR])
def test_signed_speed_bounds_are_the_extreme_eigenvalues(ora, system):
    """NE and SR: the two acoustic speeds are the smallest and largest
    eigenvalues of the flux Jacobian along e_d for every state."""
    g = 5.0 / 3.0
    rng = np.random.default_rng(17)
    for q in range(5):
        if system == NE:
            prim = np.array([[rng.uniform(0.5, 2)], [rng.uniform(-1, 1)], [rng.uniform(-1, 1)],
                             [rng.uniform(-1, 1)], [rng.uniform(0.5, 2)]])
        else:
            prim = synth.sr_samples(1, seed=200 + q, w_max=4.0)
        U = ora.prim2cons(system, g, prim)
        for d in range(3):
            ev = np.linalg.eigvals(_fd_jacobian(ora, system, g, d, U[:, 0])).real
            lm, lp = ora.wave_speeds(system, g, d, U, prim)
            assert np.abs(lp[:, 0] - ev.max()).max() <= 1e-6 * max(1.0, abs(ev).max())
            assert np.abs(lm[:, 0] - ev.min()).max() <= 1e-6 * max(1.0, abs(ev).max())


def test_mhd_speeds_without_field_are_the_hydro_speeds(ora):
    """B = 0: v_A = 0, so the fluid speeds of SRMHD are the SR acoustic ones."""
    g = 4.0 / 3.0
    prim = synth.sr_samples(300, seed=23, w_max=8.0)
    Us = ora.prim2cons(SR, g, prim)
    Um = ora.prim2cons(MHD, g, prim, np.zeros((4, 300)))
    for d in range(3):
        a_s = ora.max_speed(SR, g, d, Us, prim)
        a_m = ora.max_speed(MHD, g, d, Um, prim)
        assert np.abs(a_m[0] - a_s[0]).max() <= 1e-15
        lms, lps = ora.wave_speeds(SR, g, d, Us, prim)
        lmm, lpm = ora.wave_speeds(MHD, g, d, Um, prim)
        assert np.abs(lmm[:5] - lms).max() <= 1e-15 and np.abs(lpm[:5] - lps).max() <= 1e-15


@pytest.mark.parametrize("system", [NE, SR, MHD])
def test_roundtrip(ora, system):
    g = 4.0 / 3.0
    if system == MHD:
        prim, mag = synth.srmhd_samples(5000, seed=5)
    elif system == SR:
        prim, mag = synth.sr_samples(5000, seed=5), None
    else:
        prim = synth.sr_samples(5000, seed=5)
        prim[1:4] *= 3.0
        mag = None
    U = ora.prim2cons(system, g, prim, mag)
    P2, fail, nf = ora.cons2prim(system, g, U)
    assert nf == 0 and not fail.any()
    r = ora.backward_residual(system, g, U, P2)
    assert r.max() < 1e-13
    # forward accuracy is limited by conditioning (W up to 10-20, p/rho down to
    # 1e-4): rounding alone moves the root by ~1e-11 (SR) and ~1e-9 (MHD)
    tolp = {NE: 1e-12, SR: 2e-11, MHD: 5e-9}[system]
    assert (np.abs(P2[4] - prim[4]) / prim[4]).max() < tolp
    assert (np.abs(P2[0] - prim[0]) / prim[0]).max() < tolp


def test_sr_rest_frame_pressure_exact(ora):
    """v = 0: the recovered pressure is (gamma-1) tau exactly (W = 1)."""
    g = 4.0 / 3.0
    prim = synth.sr_samples(100, seed=9)
    prim[1:4] = 0.0
    U = ora.prim2cons(SR, g, prim)
    P2, _, _ = ora.cons2prim(SR, g, U)
    assert np.abs(P2[4] - (g - 1.0) * U[4]).max() <= 4e-16 * U[4].max()


def test_mhd_zero_field_reduces_to_hydro(ora):
    g = 4.0 / 3.0
    prim = synth.sr_samples(500, seed=13)
    Us = ora.prim2cons(SR, g, prim)
    Um = ora.prim2cons(MHD, g, prim, np.zeros((4, 500)))
    assert np.array_equal(Um[:5], Us)
    Ps, _, _ = ora.cons2prim(SR, g, Us)
    Pm, _, _ = ora.cons2prim(MHD, g, Um)
    assert np.abs(Pm - Ps).max() <= 1e-13 * np.abs(Ps).max()
    Fs = ora.flux(SR, g, 1, Us, Ps)
    Fm = ora.flux(MHD, g, 1, Um, Pm)
    assert np.abs(Fm[:5] - Fs).max() <= 1e-12 * np.abs(Fs).max()


@pytest.mark.parametrize("system", [SR, MHD])
def test_pressure_root_unique_by_scan(ora, system):
    """Brute force: f is defined on all of [0, p_hi] and changes sign exactly once."""
    g = 4.0 / 3.0
    if system == MHD:
        prim, mag = synth.srmhd_samples(60, seed=21)
    else:
        prim, mag = synth.sr_samples(60, seed=21, w_max=20.0), None
    U = ora.prim2cons(system, g, prim, mag)
    for q in range(60):
        u = U[:, q]
        pt = prim[4, q]
        phi = (g - 1) * (u[4] - (0.5 * (u[5:8] @ u[5:8]) if system == MHD else 0.0))
        grid = np.concatenate([[0.0], np.geomspace(phi * 1e-12, phi, 10000)])
        f, valid = ora.pressure_function(system, g, u, grid)
        assert valid.all()
        s = np.sign(f)
        changes = np.nonzero(s[1:] != s[:-1])[0]
        assert len(changes) == 1
        k = changes[0]
        assert grid[k] <= pt * (1 + 1e-8) and grid[k + 1] >= pt * (1 - 1e-8)


@pytest.mark.parametrize("system", [SR, MHD])
def test_unphysical_states_are_flagged(ora, system):
    g = 4.0 / 3.0
    nv = 5 if system == SR else 9
    prim, mag = synth.srmhd_samples(6, seed=2)
    if system == SR:
        mag = None
    U = ora.prim2cons(system, g, prim, mag)
    U[0, 0] = -1.0                      # negative density
    U[4, 1] = -0.5                      # negative energy
    U[1, 2] = 10 * (U[4, 2] + U[0, 2])  # momentum beyond the energy bound
    U[:, 3] = np.nan
    U[0, 4] = 0.0
    _, fail, nf = ora.cons2prim(system, g, U[:nv])
    assert list(fail[:5]) == [1, 1, 1, 1, 1] and fail[5] == 0 and nf == 5


@pytest.mark.parametrize("system", [NE, SR, MHD])
def test_llf_consistency_and_conservation(ora, system):
    g = 4.0 / 3.0
    prim, mag = synth.srmhd_samples(2, seed=4, w_max=3.0)
    if system != MHD:
        mag = None
    U = ora.prim2cons(system, g, prim, mag)
    for d in range(3):
        for sgn in (-1.0, 1.0):
            # consistency: F*(U, U).n = F(U).n
            fs = ora.llf(system, g, d, sgn, U[:, 0], prim[:, 0], U[:, 0], prim[:, 0])
            F = ora.flux(system, g, d, U[:, :1], prim[:, :1])[:, 0]
            assert np.abs(fs - sgn * F).max() <= 1e-14 * np.abs(F).max()
        # single-valued interface flux: the two sides see opposite normal fluxes
        left = ora.llf(system, g, d, 1.0, U[:, 0], prim[:, 0], U[:, 1], prim[:, 1])
        right = ora.llf(system, g, d, -1.0, U[:, 1], prim[:, 1], U[:, 0], prim[:, 0])
        assert np.abs(left + right).max() <= 1e-14 * np.abs(left).max()
