"""GPU parity of moving-split boundary sides and the double-Mach reflection (Sec. 7.4)."""
import math

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import ctx, say
from workloads import DIRICHLET, EAST, MOVING, NORTH, SLIPWALL, SOUTH, TRANSMISSIVE, WEST

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(scope="module")
def C():
    return ctx()


def gpu_residual(c, case):
    import torch
    import paper_1711_09272_amd as P
    g = P.Grid.from_case(c, case)
    r = P.residual(c, g, case.params, g.to_device(case.q0))
    torch.cuda.synchronize()
    return g.from_device(r)


def gpu_run(c, case, nsteps, t_end=0.0):
    import torch
    import paper_1711_09272_amd as P
    g = P.Grid.from_case(c, case)
    q = g.to_device(case.q0)
    st = P.step(c, g, case.params, q, nsteps, 0.0, t_end)
    torch.cuda.synchronize()
    return g.from_device(q), st


def rerr(r, r_or, sc):
    return np.array([np.abs(r[k] - r_or[k]).max() / sc[k].max() for k in range(4)])


@pytest.mark.parametrize("side", [WEST, EAST, SOUTH, NORTH])
@pytest.mark.parametrize("hi", [SLIPWALL, DIRICHLET])
@pytest.mark.parametrize("t_bc", [0.0, 0.13])
def test_moving_side_residual(C, side, hi, t_bc):
    bc = [TRANSMISSIVE] * 4
    bc[side] = MOVING
    c = workloads.smooth_random_case(37, 23, 3 + side, bc=tuple(bc), order=2, eps1=1.0)
    c.moving = {side: (0.45, 1.2, hi, workloads.conserved(1.4, 0.9, 0.1, -0.2, 0.8))}
    c.t_bc = t_bc
    r_or, sc = oracle.residual(c, with_scale=True)
    r = gpu_residual(C, c)
    assert np.all(rerr(r, r_or, sc) <= TOL64)


@pytest.mark.parametrize("ts,steps", [(0, 20), (1, 30), (2, 20)])
def test_dmr_small_steps(C, ts, steps):
    case = workloads.dmr(96, 24, t_end=0.0, time_scheme=ts)
    say(f"[dmr] 96x24 time scheme {ts}, {steps} steps")
    q_or, st_or = oracle.run(case, nsteps=steps)
    q, st = gpu_run(C, case, steps)
    err = np.abs(q - q_or).max() / np.abs(q_or).max()
    say(f"    err {err:.3e}")
    assert st["steps"] == steps and abs(st["t"] - st_or["t"]) <= 1e-13 * st_or["t"]
    assert err <= TOL64


def test_dmr_200x50_to_t_end(C):
    """The whole run to t = 0.2 on a coarse grid, against the oracle."""
    case = workloads.dmr(200, 50, t_end=0.2)
    q_or, st_or = oracle.run(case)
    q, st = gpu_run(C, case, 10 ** 6, t_end=0.2)
    err = np.abs(q - q_or).max() / np.abs(q_or).max()
    say(f"[dmr] 200x50 to t=0.2: {st['steps']} steps (oracle {st_or['steps']}), err {err:.3e}")
    assert st["t"] == 0.2 and st["steps"] == st_or["steps"] and st["nonphys"] == 0
    assert err <= TOL64


@pytest.mark.parametrize("scheme", [0, 1])
def test_dmr_full_size(C, scheme):
    """The paper's 200 x 800 grid to t = 0.2 with Roe-AM and with classical Roe:
    no non-physical state, and away from the wall the incident shock is on its
    exact line x = 1/6 + (y + 20 t)/sqrt(3) within two cells."""
    case = workloads.dmr(800, 200, t_end=0.2, scheme=scheme)
    q, st = gpu_run(C, case, 10 ** 6, t_end=0.2)
    say(f"[dmr full] scheme {scheme}: {st['steps']} steps, t {st['t']}")
    assert st["t"] == 0.2 and st["nonphys"] == 0
    for yq in (0.8, 0.9):
        j = int(yq * 200)
        y = (j + 0.5) / 200
        i_jump = int(np.argmax(np.abs(np.diff(q[0, j]))))
        x_jump = (i_jump + 1) * 4.0 / 800
        x_exact = 1.0 / 6.0 + (y + 20 * 0.2) / math.sqrt(3.0)
        assert abs(x_jump - x_exact) <= 2 * 4.0 / 800, (yq, x_jump, x_exact)


def test_moving_side_arguments(C):
    import paper_1711_09272_amd as P
    c = workloads.smooth_random_case(8, 8, 1, bc=(TRANSMISSIVE, TRANSMISSIVE, MOVING, SLIPWALL))
    g = P.Grid.from_case(C, c)
    with pytest.raises(P.RoeamError):
        g.set_moving_side(NORTH, 0.0, 0.0, SLIPWALL)  # not a moving side
    with pytest.raises(P.RoeamError):
        g.set_moving_side(SOUTH, 0.0, 0.0, TRANSMISSIVE)
    with pytest.raises(P.RoeamError):
        g.set_moving_side(SOUTH, 0.0, 0.0, DIRICHLET)  # no state
    with pytest.raises(P.RoeamError):
        g.set_moving_side(SOUTH, float("nan"), 0.0, SLIPWALL)
    g.set_moving_side(SOUTH, 0.3, 0.0, SLIPWALL)
    with pytest.raises(P.RoeamError):  # moving sides need a uniform grid
        cn = workloads.smooth_random_case(8, 8, 1, bc=(TRANSMISSIVE, TRANSMISSIVE, MOVING, SLIPWALL), nodes=True)
        P.Grid.from_case(C, cn)
