"""Python binding of libdgmi.so (argument marshalling only).

Every function mirrors the C entry point of the same name in include/dgmi.h:
tensors are torch CUDA tensors (float64 unless stated), passed as raw device
pointers; ``stream`` defaults to torch's current stream.  All computation
happens in the HIP kernels of the library; if the library is missing this
module raises on import instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgmi.so")

NEWTONIAN_EULER, SR_HYDRO, SR_MHD = 0, 1, 2
GUESS_INPUT, GUESS_PLAIN, GUESS_LEARNED, GUESS_F0 = 0, 1, 2, 3
FLAG_PLAIN_GUESS, FLAG_RECOVER_FIRST, FLAG_NO_GRAPH, FLAG_AUTOTUNE, FLAG_HLL, FLAG_POLYTROPIC = 1, 2, 4, 8, 16, 32
FLAG_ROE, FLAG_MARQUINA = 64, 128
LIMITER_NONE, LIMITER_MINMOD, LIMITER_MUSCL = 0, 1, 2
SOLUTION_ISENTROPIC_VORTEX = 1
NVARS = {NEWTONIAN_EULER: 5, SR_HYDRO: 5, SR_MHD: 9}
MLP_NUM_WEIGHTS = 4609
MLP_NUM_PARAMS = 4621

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_1609_00098_amd/build.py (hipcc, gfx950)")

_lib = ctypes.CDLL(LIB_PATH)


class DgmiError(RuntimeError):
    pass


class MeshDesc(ctypes.Structure):
    _fields_ = [("system", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("degree", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("gamma", ctypes.c_double), ("kappa", ctypes.c_double),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("degrees_host", ctypes.POINTER(ctypes.c_int32))]


_P = ctypes.c_void_p
_I32, _I64, _D = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_SIGS = {
    "dgmi_create": (_I32, [ctypes.POINTER(MeshDesc), _P, ctypes.POINTER(_P)]),
    "dgmi_destroy": (_I32, [_P]),
    "dgmi_num_nodes": (_I64, [_P]),
    "dgmi_num_vars": (_I32, [_P]),
    "dgmi_num_elements": (_I64, [_P]),
    "dgmi_elem_offsets": (_I32, [_P, _P]),
    "dgmi_elem_offsets_host": (_P, [_P]),
    "dgmi_mixed_launch_mode": (_I32, [_P, _P]),
    "dgmi_node_coords": (_I32, [_P, _P, _P]),
    "dgmi_prim2cons": (_I32, [_I32, _D, _P, _P, _P, _I64, _P]),
    "dg_rhs": (_I32, [_P, _P, _P, _P, _P]),
    "dg_step": (_I32, [_P, _P, _P, _D, _P]),
    "dg_step_noalloc": (_I32, [_P, _P, _P, _D, _P]),
    "dg_operator": (_I32, [_P, _P, _P, _P, _P]),
    "dg_rhs_checked": (_I32, [_P, _P, _P, _P, ctypes.POINTER(_I64), _P]),
    "dg_step_checked": (_I32, [_P, _P, _P, _D, ctypes.POINTER(_I64), _P]),
    "con2prim_checked": (_I32, [_I32, _D, _P, _P, _I64, _I32, _P, _D, _P, _P, _P, ctypes.POINTER(_I64), _P]),
    "dgmi_failures": (_I32, [_P, ctypes.POINTER(_I64), _P]),
    "dgmi_set_boundary": (_I32, [_P, _I32, _P, _P]),
    "dgmi_set_limiter": (_I32, [_P, _I32, _D]),
    "dgmi_set_analytic_boundary": (_I32, [_P, _I32, _I32, _P, _I32]),
    "dgmi_set_time": (_I32, [_P, _D]),
    "dgmi_max_speed": (_I32, [_P, _P, _P, _P, _P]),
    "dgmi_stable_dt": (_I32, [_P, _P, _P, _D, _P, _P]),
    "dg_step_ab3": (_I32, [_P, _P, _P, _D, _P]),
    "dgmi_get_time": (_I32, [_P, ctypes.POINTER(_D)]),
    "dg_limit": (_I32, [_P, _P, _P, _P]),
    "dgmi_limited": (_I32, [_P, ctypes.POINTER(_I64), _P]),
    "dgmi_set_fixing": (_I32, [_P, _D, _D]),
    "dgmi_fixed": (_I32, [_P, ctypes.POINTER(_I64), _P]),
    "dgmi_fix_conserved": (_I32, [_I32, _D, _D, _D, _P, _I64, _P, _P]),
    "con2prim": (_I32, [_I32, _D, _P, _P, _I64, _I32, _P, _D, _P, _P, _P, _P]),
    "dgmi_last_error": (ctypes.c_char_p, []),
    "mlp_create": (_I32, [ctypes.POINTER(_P), ctypes.c_uint64, _P]),
    "mlp_destroy": (_I32, [_P]),
    "mlp_get": (_I32, [_P, _P, _P]),
    "mlp_set": (_I32, [_P, _P, _P]),
    "mlp_features": (_I32, [_I32, _D, _P, _P, _I64, _P, _P, _P]),
    "mlp_forward": (_I32, [_P, _P, _I64, _I64, _P, _P]),
    "mlp_fit_normalization": (_I32, [_P, _P, _I64, _P, _I64, _P]),
    "mlp_grad": (_I32, [_P, _P, _I64, _P, _I64, _P, _P, _P]),
    "mlp_train_step": (_I32, [_P, _P, _I64, _P, _I64, ctypes.c_float, _P, _P]),
    "mlp_train": (_I32, [_P, _P, _P, _I64, _I64, _I32, ctypes.c_float, ctypes.c_float, _P, _P]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name, None)
    if _f is None:
        continue
    _f.restype = _res
    _f.argtypes = _args


def _check(st, what):
    if st != 0:
        msg = _lib.dgmi_last_error().decode()
        raise DgmiError(f"{what} failed ({st}): {msg}")


def _ptr(t, dtype=torch.float64, numel=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Mesh:
    """Owner of a dgmi_ctx (periodic box of affine hexahedra).  ``degrees``
    (nx*ny*nz ints in 1..7) selects the mixed-degree path."""

    def __init__(self, system, nelem, degree, gamma, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), kappa=0.0, flags=0,
                 degrees=None, stream=None):
        d = MeshDesc()
        d.system = system
        d.nx, d.ny, d.nz = nelem
        d.flags = flags
        d.gamma = gamma
        d.kappa = kappa
        d.lo[:] = list(lo)
        d.hi[:] = list(hi)
        self._deg = None
        if degrees is not None:
            import numpy as np
            self._deg = np.ascontiguousarray(degrees, dtype=np.int32)
            d.degree = -1 if degree == -1 else 0  # both select degrees_host
            d.degrees_host = self._deg.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        else:
            d.degree = degree
        h = ctypes.c_void_p()
        _check(_lib.dgmi_create(ctypes.byref(d), _stream(stream), ctypes.byref(h)), "dgmi_create")
        self.handle = h
        self.system = system
        self.gamma = gamma
        self.nelem = tuple(nelem)
        self.degree = degree
        self.nnodes = int(_lib.dgmi_num_nodes(h))
        self.nv = int(_lib.dgmi_num_vars(h))

    def close(self):
        if getattr(self, "handle", None):
            _lib.dgmi_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def elem_offsets(self):
        import numpy as np
        ne = int(_lib.dgmi_num_elements(self.handle))
        off = np.zeros(ne + 1, dtype=np.int64)
        _check(_lib.dgmi_elem_offsets(self.handle, off.ctypes.data_as(ctypes.c_void_p)), "dgmi_elem_offsets")
        return off

    def mixed_launch_mode(self):
        """(single launch?, {degree: elements per workgroup of the per-degree
        launches}) as the autotuner chose them; None for a uniform mesh."""
        import numpy as np
        epb = np.zeros(8, dtype=np.int32)
        m = int(_lib.dgmi_mixed_launch_mode(self.handle, epb.ctypes.data_as(ctypes.c_void_p)))
        if m < 0:
            return None
        return bool(m), {N: int(epb[N]) for N in range(1, 8) if epb[N] > 0}

    def elem_offsets_host(self):
        """The context's own host array of element offsets (a copy of it)."""
        import numpy as np
        ne = int(_lib.dgmi_num_elements(self.handle))
        p = _lib.dgmi_elem_offsets_host(self.handle)
        if not p:
            raise DgmiError("dgmi_elem_offsets_host: " + _lib.dgmi_last_error().decode())
        return np.ctypeslib.as_array(ctypes.cast(p, ctypes.POINTER(ctypes.c_int64)), shape=(ne + 1,)).copy()

    def node_coords(self, stream=None):
        xyz = torch.empty((3, self.nnodes), dtype=torch.float64, device="cuda")
        _check(_lib.dgmi_node_coords(self.handle, _ptr(xyz), _stream(stream)), "dgmi_node_coords")
        return xyz

    def empty_state(self):
        return torch.empty((self.nv, self.nnodes), dtype=torch.float64, device="cuda")

    def empty_prims(self):
        return torch.empty((5, self.nnodes), dtype=torch.float64, device="cuda")


def dgmi_prim2cons(system, gamma, prim, mag=None, U=None, stream=None):
    n = prim.shape[1]
    if U is None:
        U = torch.empty((NVARS[system], n), dtype=torch.float64, device=prim.device)
    _ptr(prim, numel=5 * n, name="prim")
    if system == SR_MHD:
        _ptr(mag, numel=4 * n, name="mag")
    _check(_lib.dgmi_prim2cons(system, gamma, _ptr(prim), _ptr(mag) if system == SR_MHD else None,
                               _ptr(U, numel=NVARS[system] * n, name="U"), n, _stream(stream)), "dgmi_prim2cons")
    return U


def dg_rhs(mesh, U, prim_inout, dUdt, stream=None):
    n = mesh.nnodes
    _check(_lib.dg_rhs(mesh.handle, _ptr(U, numel=mesh.nv * n, name="U"),
                       _ptr(prim_inout, numel=5 * n, name="prim_inout"),
                       _ptr(dUdt, numel=mesh.nv * n, name="dUdt"), _stream(stream)), "dg_rhs")
    return dUdt


def dg_operator(mesh, U, prim, dUdt, stream=None):
    n = mesh.nnodes
    _check(_lib.dg_operator(mesh.handle, _ptr(U, numel=mesh.nv * n, name="U"), _ptr(prim, numel=5 * n, name="prim"),
                            _ptr(dUdt, numel=mesh.nv * n, name="dUdt"), _stream(stream)), "dg_operator")
    return dUdt


def dgmi_set_boundary(mesh, direction, state_lo=None, state_hi=None):
    """Fixed exterior states (primitives, + B and Phi for SRMHD) on the two box
    faces of ``direction``; both None restores periodicity."""
    import numpy as np
    if state_lo is None and state_hi is None:
        _check(_lib.dgmi_set_boundary(mesh.handle, direction, None, None), "dgmi_set_boundary")
        return
    lo = np.ascontiguousarray(state_lo, dtype=np.float64)
    hi = np.ascontiguousarray(state_hi, dtype=np.float64)
    need = 9 if mesh.system == SR_MHD else 5
    if lo.size != need or hi.size != need:
        raise ValueError(f"states must have {need} entries")
    _check(_lib.dgmi_set_boundary(mesh.handle, direction, lo.ctypes.data_as(ctypes.c_void_p),
                                  hi.ctypes.data_as(ctypes.c_void_p)), "dgmi_set_boundary")


def dgmi_set_analytic_boundary(mesh, direction, solution, params):
    import numpy as np
    par = np.ascontiguousarray(params, dtype=np.float64)
    _check(_lib.dgmi_set_analytic_boundary(mesh.handle, direction, solution, par.ctypes.data_as(ctypes.c_void_p),
                                           par.size), "dgmi_set_analytic_boundary")


def dgmi_set_time(mesh, t):
    _check(_lib.dgmi_set_time(mesh.handle, float(t)), "dgmi_set_time")


def dgmi_get_time(mesh):
    v = _D(0.0)
    _check(_lib.dgmi_get_time(mesh.handle, ctypes.byref(v)), "dgmi_get_time")
    return float(v.value)


def dgmi_set_limiter(mesh, kind, M=0.0):
    _check(_lib.dgmi_set_limiter(mesh.handle, kind, float(M)), "dgmi_set_limiter")


def dg_limit(mesh, U, prim_inout, stream=None):
    n = mesh.nnodes
    _check(_lib.dg_limit(mesh.handle, _ptr(U, numel=mesh.nv * n, name="U"),
                         _ptr(prim_inout, numel=5 * n, name="prim_inout"), _stream(stream)), "dg_limit")
    return U


def dgmi_limited(mesh, stream=None):
    v = _I64(0)
    _check(_lib.dgmi_limited(mesh.handle, ctypes.byref(v), _stream(stream)), "dgmi_limited")
    return int(v.value)


def dgmi_set_fixing(mesh, D_min, tau_min):
    _check(_lib.dgmi_set_fixing(mesh.handle, float(D_min), float(tau_min)), "dgmi_set_fixing")


def dgmi_fixed(mesh, stream=None):
    v = _I64(0)
    _check(_lib.dgmi_fixed(mesh.handle, ctypes.byref(v), _stream(stream)), "dgmi_fixed")
    return int(v.value)


def dgmi_fix_conserved(system, gamma, D_min, tau_min, U, n_fixed=None, stream=None):
    """Fixes the columns of U ([nv, n] device tensor) in place; n_fixed: optional
    one-element int64 device tensor the number of changed columns is added to."""
    n = U.shape[1]
    _check(_lib.dgmi_fix_conserved(system, float(gamma), float(D_min), float(tau_min),
                                   _ptr(U, numel=NVARS[system] * n if system in NVARS else None, name="U"), n,
                                   _ptr(n_fixed, torch.int64, 1, "n_fixed"), _stream(stream)), "dgmi_fix_conserved")
    return U


def dgmi_max_speed(mesh, U, prim, out=None, stream=None):
    """Largest characteristic speed as a one-element device tensor."""
    n = mesh.nnodes
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device="cuda")
    _check(_lib.dgmi_max_speed(mesh.handle, _ptr(U, numel=mesh.nv * n, name="U"), _ptr(prim, numel=5 * n, name="prim"),
                               _ptr(out, numel=1, name="out"), _stream(stream)), "dgmi_max_speed")
    return out


def dgmi_stable_dt(mesh, U, prim, cfl, out=None, stream=None):
    """cfl * dx_min / lambda_max as a one-element device tensor."""
    n = mesh.nnodes
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device="cuda")
    _check(_lib.dgmi_stable_dt(mesh.handle, _ptr(U, numel=mesh.nv * n, name="U"), _ptr(prim, numel=5 * n, name="prim"),
                               float(cfl), _ptr(out, numel=1, name="out"), _stream(stream)), "dgmi_stable_dt")
    return out


def dg_step_ab3(mesh, U, prim_inout, dt, stream=None):
    n = mesh.nnodes
    _check(_lib.dg_step_ab3(mesh.handle, _ptr(U, numel=mesh.nv * n, name="U"),
                            _ptr(prim_inout, numel=5 * n, name="prim_inout"), float(dt), _stream(stream)),
           "dg_step_ab3")
    return U


def dg_step(mesh, U, prim_inout, dt, stream=None):
    n = mesh.nnodes
    _check(_lib.dg_step(mesh.handle, _ptr(U, numel=mesh.nv * n, name="U"),
                        _ptr(prim_inout, numel=5 * n, name="prim_inout"), float(dt), _stream(stream)), "dg_step")
    return U


class Con2PrimError(DgmiError):
    """A checked call found failed recoveries; ``n_failed`` holds their number."""

    def __init__(self, msg, n_failed):
        super().__init__(msg)
        self.n_failed = n_failed


_ECON2PRIM = -4


def _check_c2p(st, what, nf):
    if st == _ECON2PRIM:
        raise Con2PrimError(f"{what}: {_lib.dgmi_last_error().decode()}", int(nf.value))
    _check(st, what)


def dg_rhs_checked(mesh, U, prim_inout, dUdt, stream=None):
    """dg_rhs, then a synchronisation; raises Con2PrimError if a recovery of
    this call failed."""
    n = mesh.nnodes
    nf = _I64(0)
    _check_c2p(_lib.dg_rhs_checked(mesh.handle, _ptr(U, numel=mesh.nv * n, name="U"),
                                   _ptr(prim_inout, numel=5 * n, name="prim_inout"),
                                   _ptr(dUdt, numel=mesh.nv * n, name="dUdt"), ctypes.byref(nf), _stream(stream)),
               "dg_rhs_checked", nf)
    return dUdt


def dg_step_checked(mesh, U, prim_inout, dt, stream=None):
    n = mesh.nnodes
    nf = _I64(0)
    _check_c2p(_lib.dg_step_checked(mesh.handle, _ptr(U, numel=mesh.nv * n, name="U"),
                                    _ptr(prim_inout, numel=5 * n, name="prim_inout"), float(dt), ctypes.byref(nf),
                                    _stream(stream)), "dg_step_checked", nf)
    return U


def con2prim_checked(system, gamma, U, prim_inout, n_failed, guess=GUESS_PLAIN, mlp=None, tol=0.0, iters_out=None,
                     fail_out=None, stream=None):
    """con2prim with the failure count of this call in n_failed (one-element
    int64 device tensor); raises Con2PrimError if it is not zero."""
    n = U.shape[1]
    nf = _I64(0)
    _check_c2p(_lib.con2prim_checked(system, gamma, _ptr(U, numel=NVARS[system] * n, name="U"),
                                     _ptr(prim_inout, numel=5 * n, name="prim_inout"), n, guess,
                                     mlp.handle if mlp is not None else None, float(tol),
                                     _ptr(iters_out, torch.uint8, n, "iters_out"),
                                     _ptr(fail_out, torch.uint8, n, "fail_out"),
                                     _ptr(n_failed, torch.int64, 1, "n_failed"), ctypes.byref(nf), _stream(stream)),
               "con2prim_checked", nf)
    return prim_inout


def dg_step_noalloc(mesh, U, prim_inout, dt, stream=None):
    """dg_step with the intermediate stage states in the library's static
    device scratch (no allocation; meshes up to its capacity)."""
    n = mesh.nnodes
    _check(_lib.dg_step_noalloc(mesh.handle, _ptr(U, numel=mesh.nv * n, name="U"),
                                _ptr(prim_inout, numel=5 * n, name="prim_inout"), float(dt), _stream(stream)),
           "dg_step_noalloc")
    return U


def dgmi_failures(mesh, stream=None):
    v = ctypes.c_int64()
    _check(_lib.dgmi_failures(mesh.handle, ctypes.byref(v), _stream(stream)), "dgmi_failures")
    return int(v.value)


def con2prim(system, gamma, U, prim_inout, guess=GUESS_PLAIN, mlp=None, tol=0.0, iters_out=None, fail_out=None,
             n_failed=None, stream=None):
    n = U.shape[1]
    _check(_lib.con2prim(system, gamma, _ptr(U, numel=NVARS[system] * n, name="U"),
                         _ptr(prim_inout, numel=5 * n, name="prim_inout"), n, guess,
                         mlp.handle if mlp is not None else None, float(tol),
                         _ptr(iters_out, torch.uint8, n, "iters_out"), _ptr(fail_out, torch.uint8, n, "fail_out"),
                         _ptr(n_failed, torch.int64, 1, "n_failed"), _stream(stream)), "con2prim")
    return prim_inout


class Mlp:
    """Owner of a dgmi_mlp (5 -> 64 -> 64 -> 1 SiLU pressure-guess network)."""

    def __init__(self, seed=0, stream=None):
        h = ctypes.c_void_p()
        _check(_lib.mlp_create(ctypes.byref(h), seed, _stream(stream)), "mlp_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            _lib.mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlp_get(mlp, stream=None):
    out = torch.empty(MLP_NUM_PARAMS, dtype=torch.float32, device="cuda")
    _check(_lib.mlp_get(mlp.handle, _ptr(out, torch.float32), _stream(stream)), "mlp_get")
    return out


def mlp_set(mlp, params, stream=None):
    _check(_lib.mlp_set(mlp.handle, _ptr(params, torch.float32, MLP_NUM_PARAMS, "params"), _stream(stream)),
           "mlp_set")


def mlp_features(system, gamma, U, prim=None, feats=None, targets=None, stream=None):
    """Raw features [5][n] (float32) of U; with prim, also targets ln(p/D)."""
    n = U.shape[1]
    if feats is None:
        feats = torch.empty((5, n), dtype=torch.float32, device=U.device)
    if prim is not None and targets is None:
        targets = torch.empty(n, dtype=torch.float32, device=U.device)
    _check(_lib.mlp_features(system, float(gamma), _ptr(U, numel=NVARS[system] * n, name="U"),
                             _ptr(prim, numel=5 * n, name="prim") if prim is not None else None, n,
                             _ptr(feats, torch.float32, 5 * n, "feats"),
                             _ptr(targets, torch.float32, n, "targets") if prim is not None else None,
                             _stream(stream)), "mlp_features")
    return (feats, targets) if prim is not None else feats


def _feat(x, name="x"):
    """Feature matrix [5][ld] (or a column slice of one): pointer and ld."""
    if x.dim() != 2 or x.shape[0] != 5 or x.dtype != torch.float32 or not x.is_cuda:
        raise TypeError(f"{name} must be a float32 CUDA tensor of shape [5, batch]")
    if x.stride(1) != 1:
        raise ValueError(f"{name} columns must be contiguous")
    return ctypes.c_void_p(x.data_ptr()), x.stride(0), x.shape[1]


def _vec(t, n, name):
    if t.dim() != 1 or t.dtype != torch.float32 or not t.is_cuda or t.stride(0) != 1 or t.shape[0] != n:
        raise TypeError(f"{name} must be a contiguous float32 CUDA vector of length {n}")
    return ctypes.c_void_p(t.data_ptr())


def mlp_fit_normalization(mlp, x, t, stream=None):
    px, ld, n = _feat(x)
    _check(_lib.mlp_fit_normalization(mlp.handle, px, ld, _vec(t, n, "t"), n, _stream(stream)),
           "mlp_fit_normalization")


def mlp_forward(mlp, x, y=None, stream=None):
    """x: raw features [5][B] float32 -> predicted ln(p/D) [B]."""
    px, ld, b = _feat(x)
    if y is None:
        y = torch.empty(b, dtype=torch.float32, device=x.device)
    _check(_lib.mlp_forward(mlp.handle, px, ld, b, _vec(y, b, "y"), _stream(stream)), "mlp_forward")
    return y


def mlp_grad(mlp, x, t, grads=None, loss=None, stream=None):
    """Gradient of the mean squared error over the batch w.r.t. the 4609 weights."""
    px, ld, b = _feat(x)
    if grads is None:
        grads = torch.empty(MLP_NUM_WEIGHTS, dtype=torch.float32, device=x.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
    _check(_lib.mlp_grad(mlp.handle, px, ld, _vec(t, b, "t"), b, _vec(grads, MLP_NUM_WEIGHTS, "grads"),
                         _vec(loss, 1, "loss"), _stream(stream)), "mlp_grad")
    return grads, loss


def mlp_train_step(mlp, x, t, lr, loss=None, stream=None):
    px, ld, b = _feat(x)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
    _check(_lib.mlp_train_step(mlp.handle, px, ld, _vec(t, b, "t"), b, float(lr), _vec(loss, 1, "loss"),
                               _stream(stream)), "mlp_train_step")
    return loss


def mlp_train(mlp, x, t, batch, epochs, lr0, lr1, loss_hist=None, stream=None):
    px, ld, n = _feat(x)
    if ld != n:
        raise ValueError("mlp_train needs a contiguous [5][n] feature matrix")
    steps = (n // batch) * epochs
    if loss_hist is None:
        loss_hist = torch.empty(steps, dtype=torch.float32, device=x.device)
    _check(_lib.mlp_train(mlp.handle, px, _vec(t, n, "t"), n, batch, epochs, float(lr0), float(lr1),
                          _vec(loss_hist, steps, "loss_hist"), _stream(stream)), "mlp_train")
    return loss_hist
