"""Pins of the moving-split boundary kind and of the double-Mach reflection set-up
(Sec. 7.4) in the oracle."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads
from workloads import DIRICHLET, EAST, MOVING, NORTH, SLIPWALL, SOUTH, TRANSMISSIVE, WEST


def test_dmr_post_shock_state_satisfies_the_normal_shock_relations():
    """Mach 10 into (rho, p) = (7/5, 1), gamma = 7/5, sound speed 1: the printed
    state (8, 233/2, 33/4) from the Rankine-Hugoniot relations in exact rationals,
    and mass and momentum fluxes balance across the moving shock."""
    g, M, r1, p1 = Fraction(7, 5), 10, Fraction(7, 5), Fraction(1)
    r2 = r1 * (g + 1) * M * M / ((g - 1) * M * M + 2)
    p2 = p1 * (1 + 2 * g / (g + 1) * (M * M - 1))
    w2 = M * (1 - r1 / r2)  # shock speed M c1 = 10
    assert (r2, p2, w2) == (8, Fraction(233, 2), Fraction(33, 4))
    s = 10
    assert r1 * s == r2 * (s - w2)                               # mass
    assert p1 + r1 * s * s == p2 + r2 * (s - w2) ** 2            # momentum
    pre, post = workloads.dmr_states()
    assert post[0] == 8.0 and post[3] == 116.5
    assert math.hypot(post[1], post[2]) == pytest.approx(8.25, rel=1e-15)
    assert math.atan2(-post[2], post[1]) == pytest.approx(math.pi / 6, rel=1e-14)


def _case(bc, moving=None, seed=1):
    c = workloads.smooth_random_case(24, 13, seed, bc=bc, order=2, eps1=1.0)
    c.moving = moving
    return c


@pytest.mark.parametrize("side", [WEST, EAST, SOUTH, NORTH])
def test_moving_side_reduces_to_the_plain_kinds(side):
    """A split never reached (a below every cell) is the hi kind, a split beyond
    every cell is the side's Dirichlet state; both bitwise."""
    base = [TRANSMISSIVE] * 4
    hi_state = workloads.conserved(1.4, 0.9, 0.1, -0.2, 0.8)
    for hi in (SLIPWALL, DIRICHLET):
        bc = list(base)
        bc[side] = MOVING
        c = _case(tuple(bc), {side: (-1e9, 0.0, hi, hi_state)})
        ref_bc = list(base)
        ref_bc[side] = hi
        ref = _case(tuple(ref_bc))
        if hi == DIRICHLET:
            ref.bc_state = ref.bc_state.copy()
            ref.bc_state[side] = hi_state
        assert np.array_equal(oracle.residual(c), oracle.residual(ref))
    bc = list(base)
    bc[side] = MOVING
    c = _case(tuple(bc), {side: (1e9, 0.0, SLIPWALL, hi_state)})
    ref_bc = list(base)
    ref_bc[side] = DIRICHLET
    assert np.array_equal(oracle.residual(c), oracle.residual(_case(tuple(ref_bc))))


def test_moving_split_follows_time():
    """A split a + b t at t_bc is the fixed split a' = a + b t_bc, and it changes
    the residual when it crosses a cell centre."""
    qhi = workloads.conserved(1.4, 1.4, 0.0, 0.0, 1.0)
    c = _case((TRANSMISSIVE, TRANSMISSIVE, SLIPWALL, MOVING), {NORTH: (0.2, 1.5, DIRICHLET, qhi)})
    for t in (0.0, 0.13, 0.31):
        c.t_bc = t
        fixed = _case((TRANSMISSIVE, TRANSMISSIVE, SLIPWALL, MOVING), {NORTH: (0.2 + 1.5 * t, 0.0, DIRICHLET, qhi)})
        assert np.array_equal(oracle.residual(c), oracle.residual(fixed))
    c.t_bc = 0.0
    r0 = oracle.residual(c)
    c.t_bc = 0.31
    assert not np.array_equal(r0, oracle.residual(c))


@pytest.mark.parametrize("ts", [0, 1, 2])
def test_runs_evaluate_moving_sides_at_stage_times(ts):
    """One step of each time scheme equals the scheme composed from residuals with
    the moving sides at the abscissae of its stages (forward Euler 0; SSP-RK3
    0, 1, 1/2; the four-stage scheme 0, 1/4, 1/3, 1/2)."""
    c = workloads.dmr(96, 24, t_end=0.0, time_scheme=ts)
    c.t_bc = 0.0
    t0 = 0.0137
    q, st = oracle.run(c, nsteps=1, t0=t0)
    dt = st["dt_last"]
    q0 = c.q0

    def R(qq, t):
        c.t_bc = t
        return oracle.residual(c, q=qq)

    if ts == 0:
        ref = q0 + dt * R(q0, t0)
    elif ts == 1:
        q1 = q0 + dt * R(q0, t0)
        q2 = 0.75 * q0 + 0.25 * (q1 + dt * R(q1, t0 + dt))
        ref = (1.0 / 3.0) * q0 + (2.0 / 3.0) * (q2 + dt * R(q2, t0 + 0.5 * dt))
    else:
        a = [0.25, 1.0 / 3.0, 0.5, 1.0]
        qk = q0
        for k in range(4):
            qk = q0 + a[k] * dt * R(qk, t0 + (0.0 if k == 0 else a[k - 1] * dt))
        ref = qk
    assert np.array_equal(q, ref)


def test_dmr_incident_shock_position():
    """Away from the wall the incident shock stays on its exact line
    x = 1/6 + (y + 20 t)/sqrt(3): at t = 0.1 on a 400 x 100 grid the density
    jump at y = 0.85 lies within two cells of it (the moving top side drives it)."""
    c = workloads.dmr(400, 100, t_end=0.1)
    q, st = oracle.run(c)
    assert st["t"] == 0.1 and st["nonphys"] == 0
    j = int(0.85 * 100)
    y = (j + 0.5) / 100
    row = q[0, j]
    i_jump = int(np.argmax(np.abs(np.diff(row))))
    x_jump = (i_jump + 1) * 4.0 / 400
    x_exact = 1.0 / 6.0 + (y + 20 * 0.1) / math.sqrt(3.0)
    assert abs(x_jump - x_exact) <= 2 * 4.0 / 400, (x_jump, x_exact)
