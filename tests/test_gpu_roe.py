"""GPU parity of the Roe (eq. Roe) and Marquina fluxes (Newtonian ideal
gas) against the oracle: dg_rhs at every degree 1..7 within 1e-12
norm-wise per variable on perturbed states (the two sides of every face
differ), RK3 steps within the step bar, and the flag rules.  The Sod rows
with these fluxes run in test_gpu_limiter.py.
"""
import numpy as np
import pytest

from paper_1609_00098_amd import synth
from tests.gpu_util import normwise_err, to_dev, to_host

pytestmark = pytest.mark.gpu

NE, SR = 0, 1
LO, HI = (-0.3, 0.1, 0.0), (0.7, 1.6, 2.0)


@pytest.fixture(scope="module")
def dg():
    import torch
    assert torch.cuda.is_available()
    from paper_1609_00098_amd import dgmi
    return dgmi


def _state(ora, m, seed):
    xyz = ora.node_coords(m)
    unit = (xyz - np.array(LO)[:, None]) / (np.array(HI) - np.array(LO))[:, None]
    z = 0.02 * np.random.default_rng(seed + 100).standard_normal((5, xyz.shape[1]))
    prim = synth.fourier_random_prims(unit, seed=seed, w_max=1.5) * (1.0 + z)
    prim[1:4] *= 0.7
    return ora.prim2cons(NE, m.gamma, prim), prim


FLAGS = {"roe": "FLAG_ROE", "marquina": "FLAG_MARQUINA"}


@pytest.mark.parametrize("flux", ["roe", "marquina"])
@pytest.mark.parametrize("N", list(range(1, 8)))
def test_roe_rhs_parity(ora, dg, N, flux):
    nel = (3, 2, 2) if N <= 4 else (2, 2, 1)
    m = ora.mesh(NE, nel, N, 1.4, lo=LO, hi=HI, flux=flux)
    G = dg.Mesh(NE, nel, N, 1.4, lo=LO, hi=HI, flags=getattr(dg, FLAGS[flux]))
    U, prim = _state(ora, m, seed=30 + N)
    dUo, _, nf = ora.rhs(m, U)
    assert nf == 0
    dUd = G.empty_state()
    dg.dg_rhs(G, to_dev(U), to_dev(prim), dUd)
    assert np.all(normwise_err(to_host(dUd), dUo) <= 1e-12)
    ml = ora.mesh(NE, nel, N, 1.4, lo=LO, hi=HI)
    dUl, _, _ = ora.rhs(ml, U)
    assert np.abs(dUl - dUo).max() > 1e-6 * np.abs(dUo).max()


@pytest.mark.parametrize("flux", ["roe", "marquina"])
@pytest.mark.parametrize("N", [2, 4])
def test_roe_step_parity(ora, dg, N, flux):
    m = ora.mesh(NE, (3, 2, 2), N, 1.4, lo=LO, hi=HI, flux=flux)
    G = dg.Mesh(NE, (3, 2, 2), N, 1.4, lo=LO, hi=HI, flags=getattr(dg, FLAGS[flux]))
    U, prim = _state(ora, m, seed=40 + N)
    Lo, Po, _ = ora.rhs(m, U)
    dt = 1e-3 / max(np.abs(Lo[0] / U[0]).max(), np.abs(Lo[4] / U[4]).max())
    Uo, nf = ora.step(m, U, dt)
    assert nf == 0
    Ud = to_dev(U)
    dg.dg_step(G, Ud, to_dev(Po), dt)
    eps = np.finfo(np.float64).eps
    tol = 2e-12 * dt * np.abs(Lo).max(axis=1) + 8 * eps * np.abs(U).max(axis=1)
    assert np.all(np.abs(to_host(Ud) - Uo).max(axis=1) <= tol)


def test_roe_flag_rules(dg):
    with pytest.raises(dg.DgmiError):
        dg.Mesh(SR, (2, 2, 2), 2, 4.0 / 3.0, flags=dg.FLAG_ROE)
    with pytest.raises(dg.DgmiError):
        dg.Mesh(NE, (2, 2, 2), 2, 1.4, flags=dg.FLAG_ROE | dg.FLAG_HLL)
    with pytest.raises(dg.DgmiError):
        dg.Mesh(NE, (2, 2, 2), 2, 1.4, flags=dg.FLAG_ROE | dg.FLAG_POLYTROPIC)
    with pytest.raises(dg.DgmiError):
        dg.Mesh(NE, (2, 2, 2), 2, 1.4, flags=dg.FLAG_ROE | dg.FLAG_MARQUINA)
    with pytest.raises(dg.DgmiError):
        dg.Mesh(SR, (2, 2, 2), 2, 4.0 / 3.0, flags=dg.FLAG_MARQUINA)
