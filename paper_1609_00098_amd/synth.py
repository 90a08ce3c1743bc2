"""Seeded synthetic inputs (primitive fields and samples).

This module only draws random numbers and evaluates the analytic initial
data of the test problems at given coordinates; it holds none of the DG or
recovery arithmetic.  Both the GPU path and the CPU oracle receive their
inputs from here, and each side turns primitives into conserved variables
with its own code.

Every generator works with numpy (default) or, for large sizes, with torch
tensors on a device (``xp="torch"``); the two backends draw different random
streams for the same seed.
"""
from __future__ import annotations

import math

import numpy as np


class _Backend:
    def __init__(self, xp, seed, device=None):
        self.name = xp
        if xp == "numpy":
            self.m = np
            self.rng = np.random.default_rng(np.random.PCG64(seed))
        elif xp == "torch":
            import torch
            self.m = torch
            self.device = device or "cuda"
            self.gen = torch.Generator(device=self.device)
            self.gen.manual_seed(seed)
        else:
            raise ValueError(xp)

    def uniform(self, lo, hi, shape):
        if self.name == "numpy":
            return self.rng.uniform(lo, hi, size=shape)
        import torch
        return lo + (hi - lo) * torch.rand(shape, generator=self.gen, device=self.device, dtype=torch.float64)

    def normal(self, shape):
        if self.name == "numpy":
            return self.rng.standard_normal(size=shape)
        import torch
        return torch.randn(shape, generator=self.gen, device=self.device, dtype=torch.float64)

    def integers(self, lo, hi, shape):
        """Uniform integers in [lo, hi] inclusive."""
        if self.name == "numpy":
            return self.rng.integers(lo, hi + 1, size=shape)
        import torch
        return torch.randint(lo, hi + 1, shape, generator=self.gen, device=self.device)

    def stack(self, arrs):
        return self.m.stack(arrs)


def smooth_flow(xyz, t=0.0, amplitude=0.2, wavenumber=2.0 * math.pi, velocity=(0.2, 0.2, 0.2), pressure=1.0,
                active=(True, True, True)):
    """Advected density wave of the relativistic smooth-flow test
    (rho = 1 + A sin(k[sum_d (x_d - v_d t)]), constant v and p = 1); the same
    profile, with Newtonian constants, is the 3D Newtonian Euler workload.
    ``active`` drops collapsed directions from the phase.  Returns prim[5][n]."""
    xp = np if isinstance(xyz, np.ndarray) else _torch()
    phase = 0.0
    for d in range(3):
        if active[d]:
            phase = phase + (xyz[d] - velocity[d] * t)
    rho = 1.0 + amplitude * xp.sin(wavenumber * phase)
    ones = xp.ones_like(rho)
    return xp.stack([rho, velocity[0] * ones, velocity[1] * ones, velocity[2] * ones, pressure * ones])


def isentropic_vortex(xyz, t=0.0, beta=5.0, center=(4.0, 4.0), velocity=(1.0, 1.0, 0.0), gamma=1.4):
    """Primitives (rho, v, p) of the isentropic vortex (eq. isen_vortex) at the
    points xyz[3][n] and time t, with the isentropic pressure p = rho^gamma:
    the initial data and exact solution of the three-dimensional Newtonian
    test.  Returns prim[5][n]."""
    xp = np if isinstance(xyz, np.ndarray) else _torch()
    xt = xyz[0] - center[0] - velocity[0] * t
    yt = xyz[1] - center[1] - velocity[1] * t
    r2 = xt * xt + yt * yt
    rho = (1.0 - (gamma - 1.0) * beta ** 2 / (8.0 * gamma * math.pi ** 2) * xp.exp(1.0 - r2)) ** (1.0 / (gamma - 1.0))
    s = beta / (2.0 * math.pi) * xp.exp(0.5 * (1.0 - r2))
    vx = velocity[0] - yt * s
    vy = velocity[1] + xt * s
    return xp.stack([rho, vx, vy, velocity[2] + 0.0 * rho, rho ** gamma])


def _torch():
    import torch
    return torch


def fourier_random_prims(xyz, seed=1609, modes=8, rho_range=(0.1, 10.0), p_range=(0.01, 100.0), w_max=10.0,
                         xp="numpy", device=None):
    """Smooth random primitives on a periodic unit box.

    Five fields f_q (q = a, b, u_x, u_y, u_z), each a sum of ``modes`` sines
    c_m sin(2 pi k_m . x + phi_m), k_m in {-2..2}^3 minus 0, c_m ~ U(0.5, 1),
    phi_m ~ U(0, 2 pi), min/max-normalised over the given nodes to [-1, 1].
    rho = 10^(f_a) (in [0.1, 10]), p = 10^(2 f_b) (in [0.01, 100]),
    u = W v = sqrt(w_max^2 - 1) f_u / max|f_u| (so the largest Lorentz factor
    is exactly w_max), v = u / sqrt(1 + u^2).  Returns prim[5][n].
    """
    be = _Backend(xp, seed, device)
    m = be.m
    fields = []
    for _ in range(5):
        k = be.integers(-2, 2, (modes, 3))
        # redraw zero wave vectors deterministically
        for r in range(modes):
            while int((k[r] != 0).sum()) == 0:
                k[r] = be.integers(-2, 2, (3,))
        c = be.uniform(0.5, 1.0, (modes,))
        phi = be.uniform(0.0, 2.0 * math.pi, (modes,))
        f = 0.0
        for r in range(modes):
            arg = 2.0 * math.pi * (float(k[r][0]) * xyz[0] + float(k[r][1]) * xyz[1] + float(k[r][2]) * xyz[2])
            f = f + float(c[r]) * m.sin(arg + float(phi[r]))
        fmin, fmax = f.min(), f.max()
        fields.append(2.0 * (f - fmin) / (fmax - fmin) - 1.0)
    # rho = 10^(log-centre + half-width * f_a); p likewise
    rc = 0.5 * (math.log10(rho_range[0]) + math.log10(rho_range[1]))
    rw = 0.5 * (math.log10(rho_range[1]) - math.log10(rho_range[0]))
    pc = 0.5 * (math.log10(p_range[0]) + math.log10(p_range[1]))
    pw = 0.5 * (math.log10(p_range[1]) - math.log10(p_range[0]))
    rho = 10.0 ** (rc + rw * fields[0])
    p = 10.0 ** (pc + pw * fields[1])
    u = [fields[2], fields[3], fields[4]]
    unorm = m.sqrt(u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    scale = math.sqrt(w_max * w_max - 1.0) / float(unorm.max())
    u = [ui * scale for ui in u]
    w = m.sqrt(1.0 + u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    return m.stack([rho, u[0] / w, u[1] / w, u[2] / w, p])


def blast_wave(xyz, centre=(0.0, 0.0, 0.0), radius=0.1, rho=1.0, p_in=100.0, p_out=0.01, bfield=(10.0 ** 0.5, 0, 0),
               shell=None):
    """Spherical magnetised blast: uniform rho, v = 0, p = p_in inside r <
    radius and p_out outside, uniform B, Phi = 0.  shell=None gives a sharp
    nodal jump; shell=(r0, r1) makes ln p fall linearly from ln p_in at r0
    to ln p_out at r1 instead.  Returns (prim[5][n], mag[4][n])."""
    xp = np if isinstance(xyz, np.ndarray) else _torch()
    r2 = (xyz[0] - centre[0]) ** 2 + (xyz[1] - centre[1]) ** 2 + (xyz[2] - centre[2]) ** 2
    ones = xp.ones_like(xyz[0])
    zeros = xp.zeros_like(xyz[0])
    if shell is None:
        inside = r2 < radius * radius
        p = xp.where(inside, p_in * ones, p_out * ones)
    else:
        r0, r1 = shell
        s = (xp.sqrt(r2) - r0) / (r1 - r0)
        s = xp.clip(s, 0.0, 1.0) if xp is np else s.clamp(0.0, 1.0)
        p = xp.exp(math.log(p_in) + (math.log(p_out) - math.log(p_in)) * s)
    prim = xp.stack([rho * ones, zeros, zeros, zeros, p])
    mag = xp.stack([bfield[0] * ones, bfield[1] * ones, bfield[2] * ones, zeros])
    return prim, mag


def _unit_vectors(be, n):
    """Uniform directions on the sphere (normalised Gaussian triples)."""
    g = be.normal((3, n))
    nrm = be.m.sqrt(g[0] ** 2 + g[1] ** 2 + g[2] ** 2)
    return g / nrm


def srmhd_samples(n, seed, rho_range=(1e-3, 1e2), p_over_rho=(1e-4, 1e2), w_max=20.0, sigma_range=(1e-4, 10.0),
                  xp="numpy", device=None):
    """Random SRMHD primitive states: rho and p/rho log-uniform, ln W uniform
    in [0, ln w_max], velocity direction uniform on the sphere, magnetisation
    sigma = b^2 / rho log-uniform, field direction uniform and independent,
    |B| = sqrt(sigma rho / (1/W^2 + (Bhat.v)^2)), Phi = 0.
    Returns (prim[5][n], mag[4][n])."""
    be = _Backend(xp, seed, device)
    m = be.m
    rho = 10.0 ** be.uniform(math.log10(rho_range[0]), math.log10(rho_range[1]), (n,))
    p = rho * 10.0 ** be.uniform(math.log10(p_over_rho[0]), math.log10(p_over_rho[1]), (n,))
    W = m.exp(be.uniform(0.0, math.log(w_max), (n,)))
    vmag = m.sqrt(1.0 - 1.0 / (W * W))
    vhat = _unit_vectors(be, n)
    v = vhat * vmag
    sigma = 10.0 ** be.uniform(math.log10(sigma_range[0]), math.log10(sigma_range[1]), (n,))
    bhat = _unit_vectors(be, n)
    bv = bhat[0] * v[0] + bhat[1] * v[1] + bhat[2] * v[2]
    bmag = m.sqrt(sigma * rho / (1.0 / (W * W) + bv * bv))
    B = bhat * bmag
    prim = m.stack([rho, v[0], v[1], v[2], p])
    mag = m.stack([B[0], B[1], B[2], m.zeros_like(rho)])
    return prim, mag


def sr_samples(n, seed, rho_range=(0.1, 10.0), p_range=(0.01, 100.0), w_max=10.0, xp="numpy", device=None):
    """Random relativistic-hydro primitive states (log-uniform rho and p,
    ln W uniform in [0, ln w_max], isotropic direction).  prim[5][n]."""
    be = _Backend(xp, seed, device)
    m = be.m
    rho = 10.0 ** be.uniform(math.log10(rho_range[0]), math.log10(rho_range[1]), (n,))
    p = 10.0 ** be.uniform(math.log10(p_range[0]), math.log10(p_range[1]), (n,))
    W = m.exp(be.uniform(0.0, math.log(w_max), (n,)))
    vmag = m.sqrt(1.0 - 1.0 / (W * W))
    v = _unit_vectors(be, n) * vmag
    return m.stack([rho, v[0], v[1], v[2], p])


def mixed_degrees(nelem, seed=1610, lo=2, hi=7):
    """Per-element polynomial degree drawn uniformly from lo..hi."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    return rng.integers(lo, hi + 1, size=nelem).astype(np.int32)


def perturb(x, rel, seed):
    """x * (1 + rel * U(-1, 1)) elementwise (numpy)."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    return x * (1.0 + rel * rng.uniform(-1.0, 1.0, size=np.shape(x)))
