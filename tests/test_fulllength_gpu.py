"""Parity at the length the bench runs the configurations: the low-Mach
vortex pair (256^2 at M = 0.01 and 0.001, 1000 SSP-RK3 steps) through the
batch engine as the bench runs it, and the error growth of the Mach-20
odd-even channel (800 x 80) against the oracle over its whole run to t = 30."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import ctx, say, state_error

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    return ctx()


def test_vortex_pair_1000_steps_batched(C):
    """Both 256^2 grids of the second configuration advanced together for its
    1000 steps: each final state within 1e-12 of the oracle's (state norm),
    same step count, same final time to 1e-13; and the error curve of the M =
    0.001 grid every 100 steps through roeam_step (the same kernels)."""
    import torch
    import paper_1711_09272_amd as P
    cases = [workloads.vortex(256, 0.01), workloads.vortex(256, 0.001)]
    grids = [P.Grid.from_case(C, c) for c in cases]
    P.batch_reserve(C, sum(g.footprint() for g in grids) + (1 << 20))
    solves = [P.Solve(g, c.params, g.to_device(c.q0), 1000, 0.0, g.empty_state()) for g, c in zip(grids, cases)]
    P.batch_submit(C, solves)
    assert P.batch_run(C, -1) == 0
    for c, g, s in zip(cases, grids, solves):
        done, st, rc = P.batch_poll(C, s.ticket)
        assert done and rc == P.OK and st["steps"] == 1000
        q = g.from_device(s.q_out)
        say(f"[vortex pair] M={c.params['mach_ref']}: oracle 1000 steps ...")
        q_or, st_or = oracle.run(c, nsteps=1000)
        err = state_error(q, q_or)
        say(f"    err {err:.3e}, t {st['t']:.12e} (oracle {st_or['t']:.12e})")
        assert abs(st["t"] - st_or["t"]) <= 1e-13 * st_or["t"]
        assert err <= 1e-12
    # error growth of the M = 0.001 grid, every 100 steps
    c = cases[1]
    g = P.Grid.from_case(C, c)
    qg = g.to_device(c.q0)
    q_or, t_or, t = c.q0.copy(), 0.0, 0.0
    curve = []
    for k in range(10):
        st = P.step(C, g, c.params, qg, 100, t0=t)
        torch.cuda.synchronize()
        t = st["t"]
        q_or, st_or = oracle.run(c, nsteps=100, q=q_or, t0=t_or)
        t_or = st_or["t"]
        curve.append(state_error(g.from_device(qg), q_or))
    say(f"    M=0.001 error every 100 steps: {['%.2e' % e for e in curve]}")
    assert max(curve) <= 1e-12


def test_odd_even_error_growth_to_t30(C):
    """The third configuration to its end time t = 30 (about 2600 steps):
    within 1e-12 of the oracle for the first 50 steps (the parity bar), and the
    error curve every 100 steps after that, which the shock's odd-even
    physics may amplify, reported; both runs take the same number of steps
    and stay physical."""
    import torch
    import paper_1711_09272_amd as P
    case = workloads.odd_even()
    g = P.Grid.from_case(C, case)
    qg = g.to_device(case.q0)
    st = P.step(C, g, case.params, qg, 50, t0=0.0, t_end=case.t_end)
    torch.cuda.synchronize()
    q_or, st_or = oracle.run(case, nsteps=50, t_end=case.t_end)
    e50 = state_error(g.from_device(qg), q_or)
    say(f"[odd-even to t=30] 50 steps: err {e50:.3e}")
    assert e50 <= 1e-12 and st["steps"] == st_or["steps"] == 50
    t, t_or, steps, steps_or = st["t"], st_or["t"], 50, 50
    curve = [(50, e50)]
    while t < case.t_end:
        st = P.step(C, g, case.params, qg, 100, t0=t, t_end=case.t_end)
        torch.cuda.synchronize()
        q_or, st_or = oracle.run(case, nsteps=100, q=q_or, t0=t_or, t_end=case.t_end)
        t, t_or = st["t"], st_or["t"]
        steps += st["steps"]
        steps_or += st_or["steps"]
        curve.append((steps, state_error(g.from_device(qg), q_or)))
        assert st["nonphys"] == 0
    say(f"    error every 100 steps: {[(n, '%.2e' % e) for n, e in curve]}")
    assert steps == steps_or and t == t_or == case.t_end
    assert max(e for _, e in curve) <= 1e-6
