"""The fast and slow RMHD shock tests of tab:komissarov, read as single
shocks: their two printed states satisfy the Rankine-Hugoniot conditions
F(U_R) - F(U_L) = s (U_R - U_L) component by component with one speed s
(0.2 and 0.5 up to the four printed digits), which fixes where the shock
stands at t_final (s t_final from x = 0).  This pins the states (a
mistyped value breaks the agreement between components) and gives the GPU
runs of these tests their reference."""
import json
import os

import numpy as np

MHD = 2
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def states(ora, case):
    d = json.load(open(os.path.join(GOLD, "komissarov_states.json")))
    g = d["gamma"]
    out = []
    for side in ("left", "right"):
        s = d["tests"][case][side]
        u = np.array(s["u"])
        W = np.sqrt(1.0 + u @ u)
        prim = np.array([s["rho"], *(u / W), s["p"]])
        mag = np.array([*s["B"], 0.0])
        out.append((prim, mag, ora.prim2cons(MHD, g, prim[:, None], mag[:, None])[:, 0]))
    return g, d["tests"][case]["t_final"], out


def rh_speeds(ora, case):
    g, _, ((pl, ml, UL), (pr, mr, UR)) = states(ora, case)
    FL = ora.flux(MHD, g, 0, UL[:, None], pl[:, None])[:, 0]
    FR = ora.flux(MHD, g, 0, UR[:, None], pr[:, None])[:, 0]
    dU, dF = UR - UL, FR - FL
    keep = np.abs(dU) > 1e-9 * np.abs(UR).max()
    return dF[keep] / dU[keep]


def test_fast_shock_is_one_shock_at_speed_0_2(ora):
    s = rh_speeds(ora, "fast_shock")
    assert len(s) == 5  # D, S_x, S_y, tau, B_y jump
    assert np.all(np.abs(s - 0.2) <= 0.02 * 0.2), s


def test_slow_shock_is_one_shock_at_speed_0_5(ora):
    s = rh_speeds(ora, "slow_shock")
    assert len(s) == 5
    assert np.all(np.abs(s - 0.5) <= 1e-3 * 0.5), s
