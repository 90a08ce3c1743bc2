"""Exact solution of the Newtonian Euler Riemann problem (ideal gas, no
vacuum), the reference solution of the Riemann-problem tests (Newtonian
Riemann problems section, eq. RP).  Test infrastructure only.

The star pressure p* solves f_L(p) + f_R(p) + (u_R - u_L) = 0, where f_K is
the velocity jump across the wave separating state K from the star region:
a shock (p > p_K) by the Rankine-Hugoniot conditions, a rarefaction
(p <= p_K) by the isentropic Riemann invariant.  f is increasing in p, so
the root is found by plain bisection to the last representable bracket.
The solution is self-similar in S = (x - x_d)/t.
"""
import math

import numpy as np


def _wave_jump(p, rho, pk, ck, g):
    """f_K(p): u_K - u* for the left wave (and u* - u_K for the right)."""
    if p > pk:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        return (p - pk) * math.sqrt(A / (p + B))
    return 2.0 * ck / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)


def star_state(left, right, g):
    """(p*, u*) for left/right primitive states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)

    def f(p):
        return _wave_jump(p, rl, pl, cl, g) + _wave_jump(p, rr, pr, cr, g) + (ur - ul)

    lo, hi = 0.0, max(pl, pr)
    while f(hi) < 0.0:
        hi *= 2.0
    if f(lo) > 0.0:
        raise ValueError("vacuum is generated; not handled")
    for _ in range(2000):
        mid = lo + 0.5 * (hi - lo)
        if not (lo < mid < hi):
            break
        if f(mid) > 0.0:
            hi = mid
        else:
            lo = mid
    p = lo + 0.5 * (hi - lo)
    u = 0.5 * (ul + ur) + 0.5 * (_wave_jump(p, rr, pr, cr, g) - _wave_jump(p, rl, pl, cl, g))
    return p, u


def sample(left, right, g, x, t, x_d=0.0):
    """Primitives (rho, u, p) of the exact solution at points x and time t > 0."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    ps, us = star_state(left, right, g)
    g1 = (g - 1.0) / (2.0 * g)
    g6 = (g - 1.0) / (g + 1.0)
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros((3,) + x.shape)
    for idx, xv in np.ndenumerate(x):
        S = (xv - x_d) / t
        if S <= us:  # left of the contact
            if ps > pl:  # left shock
                sl = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + g1)
                w = (rl, ul, pl) if S <= sl else (rl * (ps / pl + g6) / (g6 * ps / pl + 1.0), us, ps)
            else:  # left rarefaction
                shl = ul - cl
                stl = us - cl * (ps / pl) ** g1
                if S <= shl:
                    w = (rl, ul, pl)
                elif S >= stl:
                    w = (rl * (ps / pl) ** (1.0 / g), us, ps)
                else:
                    u = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + S)
                    c = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - S))
                    w = (rl * (c / cl) ** (2.0 / (g - 1.0)), u, pl * (c / cl) ** (2.0 * g / (g - 1.0)))
        else:  # right of the contact
            if ps > pr:  # right shock
                sr = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + g1)
                w = (rr, ur, pr) if S >= sr else (rr * (ps / pr + g6) / (g6 * ps / pr + 1.0), us, ps)
            else:  # right rarefaction
                shr = ur + cr
                str_ = us + cr * (ps / pr) ** g1
                if S >= shr:
                    w = (rr, ur, pr)
                elif S <= str_:
                    w = (rr * (ps / pr) ** (1.0 / g), us, ps)
                else:
                    u = 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + S)
                    c = 2.0 / (g + 1.0) * (cr - 0.5 * (g - 1.0) * (ur - S))
                    w = (rr * (c / cr) ** (2.0 / (g - 1.0)), u, pr * (c / cr) ** (2.0 * g / (g - 1.0)))
        out[(slice(None),) + idx] = w
    return out
