"""Plain FP64 CPU oracle (test infrastructure only).

This package wraps ``oracle.c``: a slow, obviously-correct implementation of
the nodal DG operator, SSP-RK3 stepper and conservative-to-primitive
recovery of Kidder et al. (arXiv:1609.00098), plus the FP64 reference of the
pressure-guess MLP (``oracle/mlp.py``).  It shares no code with the GPU
library and must only be used by the tests, the smoke check and the
CPU-baseline leg of the benchmark.

Every function states the passage of the paper it follows in ``oracle.c``.
Parity status: every function is pinned by ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

NE, SR, MHD = 0, 1, 2
NVARS = {NE: 5, SR: 5, MHD: 9}


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain -O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
             "-std=c11", "-Wall", "-Wno-unused-function", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


class Mesh(ctypes.Structure):
    _fields_ = [("sys", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("deg", ctypes.c_int32 * 3), ("flux", ctypes.c_int32),
                ("gamma", ctypes.c_double), ("kappa", ctypes.c_double),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("bc", ctypes.c_int32 * 3), ("limiter", ctypes.c_int32), ("lim_M", ctypes.c_double),
                ("bc_u", (ctypes.c_double * 9) * 6), ("bc_p", (ctypes.c_double * 5) * 6),
                ("time", ctypes.c_double), ("vortex", ctypes.c_double * 6), ("eos", ctypes.c_int32),
                ("fix_D", ctypes.c_double), ("fix_tau", ctypes.c_double)]


LIMITERS = {"none": 0, "minmod": 1, "muscl": 2}


def mesh(system, nelem, degree, gamma, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), kappa=0.0, flux="llf",
         bc=None, limiter="none", M=0.0, vortex=None, time=0.0, eos="ideal", fix=None):
    """Box of nelem=(nx,ny,nz) affine elements, periodic unless ``bc`` says
    otherwise.  degree is an int or a per-direction triple; a 0 entry
    collapses that direction.  flux: "llf" (eq. LLF), "hll" (eq. HLL) or, for the
    Newtonian ideal gas, "roe" (eq. Roe) or "marquina".
    bc: {d: (state_lo, state_hi)} gives direction d fixed exterior states on
    its two box faces, each state a primitive 5-vector (rho, v, p), or for
    SRMHD a 9-vector (rho, v, p, B, Phi); {d: "vortex"} makes the exterior
    state the isentropic vortex (eq. isen_vortex, NE) with
    vortex = (beta, X0, Y0, U, V, W) at the face node and the mesh time.
    limiter: "none", "minmod" (beta 2) or "muscl" (beta 1), with the minmodB
    constant M, applied after every RK stage.  time: the time of the state
    rhs() is applied to, and of the first step of step() / evolve().
    eos: "ideal" (p = (gamma-1) rho eps) or, for NE, "polytropic"
    (p = rho^gamma).  fix: (D_min, tau_min) switches on the atmosphere floors
    and conserved-variable fixing of limited elements (SR, SRMHD; see
    fix_cons)."""
    if isinstance(degree, int):
        degree = (degree, degree, degree)
    m = Mesh()
    m.sys = system
    m.nx, m.ny, m.nz = nelem
    m.deg[:] = list(degree)
    m.flux = {"llf": 0, "hll": 1, "roe": 2, "marquina": 3}[flux]
    m.limiter = LIMITERS[limiter]
    m.lim_M = M
    m.time = time
    m.eos = {"ideal": 0, "polytropic": 1}[eos]
    if fix is not None:
        m.fix_D, m.fix_tau = fix
    if vortex is not None:
        m.vortex[:] = list(vortex)
    for d, states in (bc or {}).items():
        if isinstance(states, str):
            assert states == "vortex"
            m.bc[d] = 2
            continue
        m.bc[d] = 1
        for side, st in enumerate(states):
            st = np.asarray(st, dtype=np.float64)
            prim = st[:5].reshape(5, 1)
            mag = st[5:9].reshape(4, 1) if system == MHD else None
            u = prim2cons(system, gamma, prim, mag)[:, 0]
            m.bc_u[2 * d + side][:len(u)] = list(u)
            m.bc_p[2 * d + side][:] = list(prim[:, 0])
    m.gamma = gamma
    m.kappa = kappa
    m.lo[:] = list(lo)
    m.hi[:] = list(hi)
    return m


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    D = ctypes.POINTER(ctypes.c_double)
    I64 = ctypes.c_int64
    U8 = ctypes.POINTER(ctypes.c_uint8)
    MP = ctypes.POINTER(Mesh)
    sig = {
        "ora_num_threads": (ctypes.c_int, []),
        "ora_set_num_threads": (None, [ctypes.c_int]),
        "ora_gll": (ctypes.c_int, [ctypes.c_int, D, D]),
        "ora_legendre": (ctypes.c_double, [ctypes.c_int, ctypes.c_double]),
        "ora_diff_matrix": (ctypes.c_int, [ctypes.c_int, D, D]),
        "ora_lagrange_matrix": (ctypes.c_int, [ctypes.c_int, D, ctypes.c_int, D, D]),
        "ora_prim2cons": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, I64, D, D, D]),
        "ora_cons2prim": (I64, [ctypes.c_int, ctypes.c_double, I64, D, D, U8]),
        "ora_c2p_pressure_function": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, D, I64, D, D, U8]),
        "ora_c2p_f_points": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, I64, D, D, D, U8]),
        "ora_backward_residual": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, I64, D, D, D]),
        "ora_flux": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_int, I64, D, D, D]),
        "ora_max_speed": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_int, I64, D, D, D]),
        "ora_wave_speeds": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_int, I64, D, D, D, D]),
        "ora_llf": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double, D, D, D, D, D]),
        "ora_num_nodes": (I64, [MP]),
        "ora_node_coords": (ctypes.c_int, [MP, D]),
        "ora_rhs": (I64, [MP, D, D, D]),
        "ora_rhs_elements": (ctypes.c_int, [MP, D, D, I64, ctypes.POINTER(I64), D]),
        "ora_rhs_weak": (I64, [MP, D, D]),
        "ora_rk3_combine": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, I64, D, D, D, D]),
        "ora_step": (I64, [MP, D, ctypes.c_double]),
        "ora_evolve": (I64, [MP, D, ctypes.c_double, I64]),
        "ora_l1_error": (ctypes.c_double, [MP, ctypes.c_int, D, D]),
        "ora_integrate": (ctypes.c_int, [MP, ctypes.c_int, D, D]),
        "ora_hll": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double, D, D, D, D, D]),
        "ora_mixed_num_nodes": (I64, [ctypes.c_int, ctypes.POINTER(ctypes.c_int32)]),
        "ora_mixed_node_coords": (ctypes.c_int, [MP, ctypes.POINTER(ctypes.c_int32), D]),
        "ora_rhs_mixed": (I64, [MP, ctypes.POINTER(ctypes.c_int32), D, D, D]),
        "ora_mixed_integrate": (ctypes.c_int, [MP, ctypes.POINTER(ctypes.c_int32), ctypes.c_int, D, D]),
        "ora_step_mixed": (I64, [MP, ctypes.POINTER(ctypes.c_int32), D, ctypes.c_double]),
        "ora_minmodB": (ctypes.c_double, [ctypes.c_double] * 5),
        "ora_limit": (I64, [MP, D]),
        "ora_limiter_moments": (ctypes.c_int, [MP, D, D, U8]),
        "ora_isentropic_vortex": (ctypes.c_int, [ctypes.c_double, D, I64, D, ctypes.c_double, D]),
        "ora_max_char_speed": (ctypes.c_double, [MP, D]),
        "ora_roe": (ctypes.c_int, [ctypes.c_double, ctypes.c_int, ctypes.c_double, D, D, D, D, D]),
        "ora_marquina": (ctypes.c_int, [ctypes.c_double, ctypes.c_int, ctypes.c_double, D, D, D, D, D]),
        "ora_min_node_spacing": (ctypes.c_double, [MP]),
        "ora_stable_dt": (ctypes.c_double, [MP, D, ctypes.c_double]),
        "ora_evolve_ab3": (I64, [MP, D, ctypes.c_double, I64]),
        "ora_limit_counts": (ctypes.c_int, [MP, D, ctypes.POINTER(I64)]),
        "ora_limit_mixed": (I64, [MP, ctypes.POINTER(ctypes.c_int32), D, ctypes.POINTER(I64)]),
        "ora_evolve_ab3_mixed": (I64, [MP, ctypes.POINTER(ctypes.c_int32), D, ctypes.c_double, I64]),
        "ora_stable_dt_mixed": (ctypes.c_double, [MP, ctypes.POINTER(ctypes.c_int32), D, ctypes.c_double]),
        "ora_fix_cons": (I64, [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, I64, D]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def num_threads():
    return int(_load().ora_num_threads())


def set_num_threads(n):
    _load().ora_set_num_threads(int(n))


# ----------------------------------------------------------------- tables
def gll(N):
    x = np.zeros(N + 1)
    w = np.zeros(N + 1)
    if _load().ora_gll(N, _p(x), _p(w)) != 0:
        raise ValueError("bad degree")
    return x, w


def legendre(N, x):
    return _load().ora_legendre(N, float(x))


def diff_matrix(N):
    x, _ = gll(N)
    D = np.zeros((N + 1) * (N + 1))
    _load().ora_diff_matrix(N, _p(x), _p(D))
    return D.reshape(N + 1, N + 1)


def lagrange_matrix(xfrom, yto):
    xfrom = _c(xfrom)
    yto = _c(yto)
    out = np.zeros(len(yto) * len(xfrom))
    _load().ora_lagrange_matrix(len(xfrom), _p(xfrom), len(yto), _p(yto), _p(out))
    return out.reshape(len(yto), len(xfrom))


# --------------------------------------------------------------- pointwise
def prim2cons(system, gamma, prim, mag=None):
    prim = _c(prim)
    n = prim.shape[1]
    nv = NVARS[system]
    U = np.zeros((nv, n))
    magp = None
    if system == MHD:
        mag = _c(mag)
        magp = _p(mag)
    _load().ora_prim2cons(system, gamma, n, _p(prim), magp, _p(U))
    return U


def cons2prim(system, gamma, U):
    U = _c(U)
    n = U.shape[1]
    prim = np.zeros((5, n))
    fail = np.zeros(n, dtype=np.uint8)
    nf = _load().ora_cons2prim(system, gamma, n, _p(U), _p(prim),
                               fail.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    return prim, fail, nf


def pressure_function(system, gamma, u1, p):
    u1 = _c(u1)
    p = _c(p)
    f = np.zeros_like(p)
    valid = np.zeros(len(p), dtype=np.uint8)
    _load().ora_c2p_pressure_function(system, gamma, _p(u1), len(p), _p(p), _p(f),
                                      valid.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    return f, valid.astype(bool)


def pressure_function_points(system, gamma, U, p):
    """f(p[q]) of state q for every point (one trial pressure per point)."""
    U = _c(U)
    p = _c(p)
    f = np.zeros(U.shape[1])
    valid = np.zeros(U.shape[1], dtype=np.uint8)
    _load().ora_c2p_f_points(system, gamma, U.shape[1], _p(U), _p(p), _p(f),
                             valid.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    return f, valid.astype(bool)


def backward_residual(system, gamma, U, prim):
    U = _c(U)
    prim = _c(prim)
    r = np.zeros(U.shape[1])
    _load().ora_backward_residual(system, gamma, U.shape[1], _p(U), _p(prim), _p(r))
    return r


def flux(system, gamma, d, U, prim):
    U = _c(U)
    prim = _c(prim)
    F = np.zeros_like(U)
    _load().ora_flux(system, gamma, d, U.shape[1], _p(U), _p(prim), _p(F))
    return F


def max_speed(system, gamma, d, U, prim):
    U = _c(U)
    prim = _c(prim)
    a = np.zeros_like(U)
    _load().ora_max_speed(system, gamma, d, U.shape[1], _p(U), _p(prim), _p(a))
    return a


def wave_speeds(system, gamma, d, U, prim):
    """Signed speed bounds (lm, lp), each [nv][n], of every component along +e_d."""
    U = _c(U)
    prim = _c(prim)
    lm = np.zeros_like(U)
    lp = np.zeros_like(U)
    _load().ora_wave_speeds(system, gamma, d, U.shape[1], _p(U), _p(prim), _p(lm), _p(lp))
    return lm, lp


def llf(system, gamma, d, sgn, ui, pi, ue, pe):
    out = np.zeros(NVARS[system])
    _load().ora_llf(system, gamma, d, sgn, _p(_c(ui)), _p(_c(pi)), _p(_c(ue)), _p(_c(pe)), _p(out))
    return out


def hll(system, gamma, d, sgn, ui, pi, ue, pe):
    out = np.zeros(NVARS[system])
    _load().ora_hll(system, gamma, d, sgn, _p(_c(ui)), _p(_c(pi)), _p(_c(ue)), _p(_c(pe)), _p(out))
    return out


# -------------------------------------------------------------------- mesh
def num_nodes(m):
    return int(_load().ora_num_nodes(ctypes.byref(m)))


def node_coords(m):
    n = num_nodes(m)
    xyz = np.zeros((3, n))
    _load().ora_node_coords(ctypes.byref(m), _p(xyz))
    return xyz


def rhs(m, U):
    """Returns (dUdt, prims, n_failed)."""
    U = _c(U)
    n = U.shape[1]
    prim = np.zeros((5, n))
    dU = np.zeros_like(U)
    nf = _load().ora_rhs(ctypes.byref(m), _p(U), _p(prim), _p(dU))
    if nf < 0:
        raise ValueError("bad mesh")
    return dU, prim, int(nf)


def rhs_elements(m, U, prim, elems):
    U = _c(U)
    prim = _c(prim)
    elems = _c(elems, np.int64)
    npe = num_nodes(m) // (m.nx * m.ny * m.nz)
    out = np.zeros((U.shape[0], len(elems) * npe))
    rc = _load().ora_rhs_elements(ctypes.byref(m), _p(U), _p(prim), len(elems),
                                  elems.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p(out))
    if rc != 0:
        raise ValueError("bad element list")
    return out


def rhs_weak(m, U):
    U = _c(U)
    dU = np.zeros_like(U)
    _load().ora_rhs_weak(ctypes.byref(m), _p(U), _p(dU))
    return dU


def roe(gamma, d, sgn, ui, pi, ue, pe):
    out = np.zeros(5)
    _load().ora_roe(gamma, d, sgn, _p(_c(ui)), _p(_c(pi)), _p(_c(ue)), _p(_c(pe)), _p(out))
    return out


def marquina(gamma, d, sgn, ui, pi, ue, pe):
    out = np.zeros(5)
    _load().ora_marquina(gamma, d, sgn, _p(_c(ui)), _p(_c(pi)), _p(_c(ue)), _p(_c(pe)), _p(out))
    return out


def isentropic_vortex(gamma, params, xyz, t):
    """Primitives of eq. isen_vortex (params = beta, X0, Y0, U, V, W) at the
    points xyz[3][n] and time t."""
    xyz = _c(xyz)
    n = xyz.shape[1]
    par = _c(params)
    out = np.zeros((5, n))
    _load().ora_isentropic_vortex(gamma, _p(par), n, _p(xyz), t, _p(out))
    return out


def minmodB(a1, a2, a3, M=0.0, dx=1.0):
    return float(_load().ora_minmodB(a1, a2, a3, M, dx))


def limit(m, U):
    """Returns (limited copy of U, number of limited element components)."""
    U = _c(U).copy()
    n = _load().ora_limit(ctypes.byref(m), _p(U))
    if n < 0:
        raise ValueError("bad mesh")
    return U, int(n)


def limit_counts(m, U):
    """Returns (limited copy of U, limited element components, nodes changed
    by the conserved-variable fixing)."""
    U = _c(U).copy()
    counts = np.zeros(2, dtype=np.int64)
    if _load().ora_limit_counts(ctypes.byref(m), _p(U), counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))) != 0:
        raise ValueError("bad mesh")
    return U, int(counts[0]), int(counts[1])


def fix_cons(system, gamma, U, D_min, tau_min):
    """Atmosphere floors and conserved-variable fixing (section on unphysical
    conservative variables) of every column of U ([nv, n]); returns (fixed
    copy, number of columns changed)."""
    U = _c(U).copy()
    n = _load().ora_fix_cons(system, gamma, D_min, tau_min, U.shape[1], _p(U))
    if n < 0:
        raise ValueError("bad arguments")
    return U, int(n)


def limiter_moments(m, U):
    """Per element [10][nv]: mean, Legendre slope coefficients c_x, c_y, c_z,
    face means -x, +x, -y, +y, -z, +z; and the unphysical-node flag."""
    U = _c(U)
    ne = m.nx * m.ny * m.nz
    out = np.zeros((ne, 10, U.shape[0]))
    bad = np.zeros(ne, dtype=np.uint8)
    if _load().ora_limiter_moments(ctypes.byref(m), _p(U), _p(out),
                                   bad.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))) != 0:
        raise ValueError("bad mesh")
    return out, bad


def rk3_combine(stage, dt, Un, Uprev, L):
    Un, Uprev, L = _c(Un), _c(Uprev), _c(L)
    out = np.zeros_like(Un)
    if _load().ora_rk3_combine(stage, dt, Un.size, _p(Un), _p(Uprev), _p(L), _p(out)) != 0:
        raise ValueError("bad stage")
    return out


def step(m, U, dt):
    U = _c(U).copy()
    nf = _load().ora_step(ctypes.byref(m), _p(U), dt)
    return U, int(nf)


def evolve(m, U, dt, nsteps):
    U = _c(U).copy()
    nf = _load().ora_evolve(ctypes.byref(m), _p(U), dt, nsteps)
    return U, int(nf)


def max_char_speed(m, U):
    return float(_load().ora_max_char_speed(ctypes.byref(m), _p(_c(U))))


def min_node_spacing(m):
    return float(_load().ora_min_node_spacing(ctypes.byref(m)))


def stable_dt(m, U, cfl):
    return float(_load().ora_stable_dt(ctypes.byref(m), _p(_c(U)), cfl))


def evolve_ab3(m, U, dt, nsteps):
    U = _c(U).copy()
    nf = _load().ora_evolve_ab3(ctypes.byref(m), _p(U), dt, nsteps)
    if nf < 0:
        raise ValueError("bad mesh")
    return U, int(nf)


def l1_error(m, a, b):
    a, b = _c(a), _c(b)
    return float(_load().ora_l1_error(ctypes.byref(m), a.shape[0], _p(a), _p(b)))


def integrate(m, q):
    q = _c(q)
    out = np.zeros(q.shape[0])
    _load().ora_integrate(ctypes.byref(m), q.shape[0], _p(q), _p(out))
    return out


# ------------------------------------------------------- mixed degrees
def _deg(deg):
    d = np.ascontiguousarray(deg, dtype=np.int32)
    return d, d.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def mixed_num_nodes(deg):
    d, dp = _deg(deg)
    return int(_load().ora_mixed_num_nodes(len(d), dp))


def mixed_node_coords(m, deg):
    d, dp = _deg(deg)
    n = mixed_num_nodes(d)
    xyz = np.zeros((3, n))
    if _load().ora_mixed_node_coords(ctypes.byref(m), dp, _p(xyz)) != 0:
        raise ValueError("bad degrees")
    return xyz


def rhs_mixed(m, deg, U):
    """Mixed-degree operator (mortar of the max degree on unequal faces)."""
    d, dp = _deg(deg)
    U = _c(U)
    prim = np.zeros((5, U.shape[1]))
    dU = np.zeros_like(U)
    nf = _load().ora_rhs_mixed(ctypes.byref(m), dp, _p(U), _p(prim), _p(dU))
    if nf < 0:
        raise ValueError("bad degrees")
    return dU, prim, int(nf)


def mixed_integrate(m, deg, q):
    d, dp = _deg(deg)
    q = _c(q)
    out = np.zeros(q.shape[0])
    _load().ora_mixed_integrate(ctypes.byref(m), dp, q.shape[0], _p(q), _p(out))
    return out


def step_mixed(m, deg, U, dt):
    d, dp = _deg(deg)
    U = _c(U).copy()
    nf = _load().ora_step_mixed(ctypes.byref(m), dp, _p(U), dt)
    return U, int(nf)


def limit_mixed(m, deg, U):
    """Limiter on a mixed-degree mesh: (limited copy of U, limited element
    components, nodes changed by the fixing)."""
    d, dp = _deg(deg)
    U = _c(U).copy()
    counts = np.zeros(2, dtype=np.int64)
    r = _load().ora_limit_mixed(ctypes.byref(m), dp, _p(U), counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if r < 0:
        raise ValueError("bad mesh")
    return U, int(counts[0]), int(counts[1])


def evolve_ab3_mixed(m, deg, U, dt, nsteps):
    """nsteps third-order Adams-Bashforth steps on a mixed-degree mesh (the
    first two are SSP-RK3 steps); returns (U, failed recoveries)."""
    d, dp = _deg(deg)
    U = _c(U).copy()
    nf = _load().ora_evolve_ab3_mixed(ctypes.byref(m), dp, _p(U), dt, nsteps)
    if nf < 0:
        raise ValueError("bad mesh")
    return U, int(nf)


def stable_dt_mixed(m, deg, U, cfl):
    d, dp = _deg(deg)
    return float(_load().ora_stable_dt_mixed(ctypes.byref(m), dp, _p(_c(U)), cfl))
