"""Pins of the supersonic corner (Sec. 7.3) and of the split side it runs on.

The case is read as the block x > 0.05 whose west side is the step's slip wall
below the corner and the post-shock inflow above it (the inflow is supersonic,
so the channel upstream of the corner stays uniform).  A split side whose lower
kind is a wall must reduce to the plain kinds when the split lies beyond the
side; the states printed in the paper must satisfy the Rankine-Hugoniot
relations of a shock moving into gas at rest; a coarse run must carry the
incident shock at the exact speed.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from workloads import DIRICHLET, EAST, MOVING, NORTH, SLIPWALL, SOUTH, TRANSMISSIVE, WEST

G = 1.4


def _case(side, kind, **kw):
    bc = [TRANSMISSIVE] * 4
    bc[side] = kind
    return workloads.smooth_random_case(23, 17, 30 + side, bc=tuple(bc), order=2, eps1=1.0, mach_ref=0.3, **kw)


@pytest.mark.parametrize("side", [WEST, EAST, SOUTH, NORTH])
def test_wall_below_a_split_beyond_the_side_is_a_slip_wall(side):
    c_wall = _case(side, SLIPWALL)
    c_split = _case(side, MOVING)
    c_split.moving = {side: (math.inf, 0.0, DIRICHLET, workloads.conserved(G, 1.0, 0.1, 0.2, 0.9), SLIPWALL)}
    assert np.array_equal(oracle.residual(c_split), oracle.residual(c_wall))


@pytest.mark.parametrize("side", [WEST, EAST, SOUTH, NORTH])
def test_state_above_a_split_before_the_side_is_dirichlet(side):
    q_hi = workloads.conserved(G, 1.3, -0.2, 0.1, 0.8)
    c_dir = _case(side, DIRICHLET)
    c_dir.bc_state[side] = q_hi
    c_split = _case(side, MOVING)
    c_split.moving = {side: (-math.inf, 0.0, DIRICHLET, q_hi, SLIPWALL)}
    assert np.array_equal(oracle.residual(c_split), oracle.residual(c_dir))


def test_split_with_wall_below_matches_its_two_halves():
    """On a west side split at y = 0.5 (wall below, Dirichlet above), the cells
    of the lower half see the wall grid's residual and those of the upper half
    the Dirichlet grid's, away from the rows whose stencils cross the split."""
    q_hi = workloads.conserved(G, 1.3, 0.4, 0.1, 0.8)
    c_split = _case(WEST, MOVING)
    ny = c_split.ny
    a = (ny // 2) * c_split.dy
    c_split.moving = {WEST: (a, 0.0, DIRICHLET, q_hi, SLIPWALL)}
    c_wall = _case(WEST, SLIPWALL)
    c_dir = _case(WEST, DIRICHLET)
    c_dir.bc_state[WEST] = q_hi
    r = oracle.residual(c_split)
    h = ny // 2
    assert np.array_equal(r[:, : h - 2, :4], oracle.residual(c_wall)[:, : h - 2, :4])
    assert np.array_equal(r[:, h + 2:, :4], oracle.residual(c_dir)[:, h + 2:, :4])


def test_paper_corner_states_satisfy_rankine_hugoniot():
    """Sec. 7.3 prints (7.04108, 4.07794, 0, 30.05942) behind the shock and
    (1.4, 0, 0, 1) ahead of it: with the shock speed W from the mass balance,
    momentum and energy balance to the printed digits, W is 5.09 (the Mach-5.09
    shock of this test) and the inflow is supersonic."""
    pre, post = workloads.corner_states()
    rR, uR, _, pR = pre
    rL, uL, _, pL = post
    W = rL * uL / (rL - rR)
    assert abs(W - 5.09) < 5e-5
    assert abs(W / math.sqrt(G * pR / rR) - 5.09) < 5e-5
    mom = rL * uL * (uL - W) + pL - (rR * uR * (uR - W) + pR)
    EL = pL / (G - 1) + 0.5 * rL * uL * uL
    ER = pR / (G - 1)
    en = (EL + pL) * uL - W * EL - ((ER + pR) * uR - W * ER)
    assert abs(mom) < 1e-5 * pL and abs(en) < 1e-5 * (EL + pL) * uL
    assert uL > math.sqrt(G * pL / rL)


def _corner_checks(c, q):
    """Equal-area position of the incident shock on the top row (which the
    corner's expansion has not reached by t = 0.155) and the mass balance (the
    wall passes no mass and nothing has left the block yet, so the mass gained
    is the inflow rho_L u_L times the channel height 1/2 times t)."""
    pre, post = workloads.corner_states()
    n = c.ny
    x_exact = 0.05 + post[0] * post[1] / (post[0] - pre[0]) * 0.155
    x_eq = 0.05 + (q[0, n - 1] - pre[0]).sum() / n / (post[0] - pre[0])
    gain = (q[0].sum() - c.q0[0].sum()) / n ** 2
    inflow = post[0] * post[1] * 0.5 * 0.155
    return (x_eq - x_exact) * n, gain / inflow - 1.0


@pytest.mark.parametrize("kw", [dict(), dict(eps1=1.0), dict(variant=oracle.V_NO_EQ92),
                                dict(order=2, time_scheme=1, eps1=1.0)],
                         ids=["roeam", "roeam_eps1", "roeam_no_eq92", "roeam_muscl_rk3"])
def test_corner_coarse_run(kw):
    """76 x 80 cells to t = 0.155 (Fig. 8 d-f and a MUSCL run): physical
    throughout, the incident shock within 0.1 cell of x = 0.05 + W t, the mass
    gain equal to the inflow within 1e-4 (the start at the corner is a
    transient)."""
    c = workloads.corner(80, **kw)
    q, st = oracle.run(c)
    assert st["t"] == 0.155 and st["nonphys"] == 0
    off, dm = _corner_checks(c, q)
    assert abs(off) <= 0.1 and abs(dm) <= 1e-4, (off, dm)


@pytest.mark.parametrize("kw", [dict(scheme=oracle.SCHEME_ROE), dict(scheme=oracle.SCHEME_ROE_HARTEN, eps_lambda=0.2),
                                dict(variant=oracle.V_XI_EQ46)], ids=["roe", "roe_harten_0.2", "roeam_xi_eq46"])
def test_corner_without_velocity_positivity_fails(kw):
    """The expansion around the corner is close to vacuum (the post-shock flow
    at Mach 1.67 turns by 90 degrees).  Without the velocity-positivity
    condition of Eq. (86) -- classical Roe, Roe with Harten's fix at 0.2, and
    Roe-AM with xi of Eq. (46) -- the run reaches a negative density or
    pressure within its first 25 steps (at any CFL number tried, 0.05 to 0.4,
    and at either order); Roe-AM with it runs through."""
    c = workloads.corner(80, **kw)
    with pytest.raises(oracle.NonPhysical):
        oracle.run(c, nsteps=40)
