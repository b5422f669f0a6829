"""Batched and continuously batched solves on the GPU: every result must be
bitwise equal to the same solve run alone through roeam_step (same kernels,
same tile shape), whatever else shares the launches, and a solve that goes
non-physical must not disturb the others."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import ctx, say, state_error
from workloads import DIRICHLET, PERIODIC, SLIPWALL, TRANSMISSIVE

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    return ctx()


def family():
    """Uneven grids, all boundary kinds, both orders, both time schemes and
    both precisions (so several work-list groups run side by side)."""
    rng = np.random.Generator(np.random.PCG64(workloads.SEED_BASE + 50))
    cases = []
    for n, steps in ((40, 9), (67, 14), (33, 5), (90, 11)):
        cases.append(workloads.bump_case(n, rng, steps))
    c = workloads.smooth_random_case(45, 29, 3, bc=(DIRICHLET, TRANSMISSIVE, SLIPWALL, SLIPWALL), nodes=True,
                                     order=2, eps1=1.0, mach_ref=0.05)
    c.nsteps = 7
    cases.append(c)
    c = workloads.sod(nx=120, ny=3)  # forward Euler, first order, stops at t_end
    c.t_end = 0.05
    cases.append(c)
    c = workloads.bump_case(50, rng, 8)
    c.params["precision"] = 1
    cases.append(c)
    c = workloads.bump_case(37, rng, 6)
    c.params["time_scheme"] = 2  # the four-stage scheme in its own group
    cases.append(c)
    return cases


def run_alone(C, case):
    import torch
    import paper_1711_09272_amd as P
    g = P.Grid.from_case(C, case)
    g.set_tile_shape(0)
    q = g.to_device(case.q0)
    st = P.step(C, g, case.params, q, case.nsteps, 0.0, case.t_end)
    torch.cuda.synchronize()
    return g.from_device(q), st


def submit_all(C, cases, grids=None):
    import paper_1711_09272_amd as P
    grids = grids or [P.Grid.from_case(C, c) for c in cases]
    solves = [P.Solve(g, c.params, P.padded(g, c.q0), c.nsteps, c.t_end) for g, c in zip(grids, cases)]
    P.batch_submit(C, solves)
    return grids, solves


def collect(C, solves):
    import paper_1711_09272_amd as P
    out = []
    for s in solves:
        done, st, rc = P.batch_poll(C, s.ticket)
        assert done, s.ticket
        out.append((s.q_out[:, :, : s.grid.nx].copy(), st, rc))
    return out


def test_batch_equals_single_runs(C):
    import paper_1711_09272_amd as P
    cases = family()
    P.batch_reserve(C, 256 << 20)
    say(f"[batch] {len(cases)} solves in one batch")
    _, solves = submit_all(C, cases)
    assert P.batch_run(C, -1) == 0
    res = collect(C, solves)
    for c, (q, st, rc) in zip(cases, res):
        qa, sta = run_alone(C, c)
        say(f"    {c.name}: steps {st['steps']} t {st['t']:.4e}")
        assert rc == P.OK and st["steps"] == sta["steps"] and st["t"] == sta["t"]
        assert np.array_equal(q, qa), c.name


def test_poll_without_handoff_then_one_leave(C):
    """The bench's polling loop: finite batch_run calls (the outputs are still
    being written on the library's stream when a poll first reports them
    done), batch_poll(..., leave=False) for every solve and one ctx.leave()
    per loop that saw a solve finish; the outputs read on torch's stream
    afterwards are bitwise those of the solves run alone."""
    import paper_1711_09272_amd as P
    cases = family()[:4]
    P.batch_reserve(C, 128 << 20)
    P.batch_configure(C, graph_iters=2)
    try:
        grids = [P.Grid.from_case(C, c) for c in cases]
        solves = [P.Solve(g, c.params, g.to_device(c.q0), c.nsteps, c.t_end, g.empty_state())
                  for g, c in zip(grids, cases)]
        P.batch_submit(C, solves)
        fin = {}
        for _ in range(200):
            if len(fin) == len(solves):
                break
            P.batch_run(C, 2)
            n0 = len(fin)
            for s in solves:
                if s.ticket not in fin:
                    done, st, rc = P.batch_poll(C, s.ticket, leave=False)
                    if done:
                        fin[s.ticket] = (st, rc)
            if len(fin) > n0:
                C.leave()
                for s in solves:
                    if s.ticket in fin and len(fin[s.ticket]) == 2:
                        fin[s.ticket] = fin[s.ticket] + (s.q_out[:, :, : s.grid.nx].clone(),)
        assert len(fin) == len(solves)
        assert P.batch_run(C, -1) == 0
    finally:
        P.batch_configure(C)
    say(f"[batch poll, one hand-off] {len(cases)} solves")
    for c, s in zip(cases, solves):
        st, rc, q = fin[s.ticket]
        qa, sta = run_alone(C, c)
        assert rc == P.OK and st["steps"] == sta["steps"] and st["t"] == sta["t"]
        assert np.array_equal(q.cpu().numpy(), qa), c.name


def test_batch_with_transported_scalars(C):
    """Grids with none, one and two scalars in one batch (three work-list
    groups per scheme): bitwise the solves run alone, and a two-scalar member
    within 1e-12 of the oracle."""
    import paper_1711_09272_amd as P
    rng = np.random.Generator(np.random.PCG64(workloads.SEED_BASE + 51))
    cases = [workloads.add_scalars(workloads.bump_case(40, rng, 9), 1, seed=1),
             workloads.add_scalars(workloads.smooth_random_case(45, 29, 3, bc=(DIRICHLET, TRANSMISSIVE, SLIPWALL,
                                                                                SLIPWALL), nodes=True, order=2,
                                                                eps1=1.0, mach_ref=0.05), 2, seed=2,
                                   k_bc=np.array([[0.5, 1.5]] * 4)),
             workloads.bump_case(33, rng, 5),
             workloads.add_scalars(workloads.bump_case(37, rng, 6), 2, seed=3, mode="smooth")]
    cases[1].nsteps = 7
    cases[3].params["time_scheme"] = 2
    P.batch_reserve(C, 128 << 20)
    say(f"[batch scalars] {len(cases)} solves, scalars {[c.q0.shape[0] - 4 for c in cases]}")
    _, solves = submit_all(C, cases)
    assert P.batch_run(C, -1) == 0
    res = collect(C, solves)
    for c, (q, st, rc) in zip(cases, res):
        qa, sta = run_alone(C, c)
        assert rc == P.OK and st["steps"] == sta["steps"] and st["t"] == sta["t"]
        assert np.array_equal(q, qa), c.name
    q_or, st_or = oracle.run(cases[1])
    assert res[1][1]["steps"] == st_or["steps"] and state_error(res[1][0], q_or) <= 1e-12


def test_batch_member_matches_oracle(C):
    import paper_1711_09272_amd as P
    cases = family()[:2]
    P.batch_reserve(C, 64 << 20)
    _, solves = submit_all(C, cases)
    P.batch_run(C, -1)
    for c, (q, st, rc) in zip(cases, collect(C, solves)):
        q_or, st_or = oracle.run(c)
        assert st["steps"] == st_or["steps"]
        assert state_error(q, q_or) <= 1e-12


def test_continuous_admission_and_arena_pressure(C):
    """Solves submitted while others run join at the next iteration; an arena
    that holds only two solves at a time still completes every solve, and each
    result is bitwise the solve run alone."""
    import paper_1711_09272_amd as P
    cases = family()
    grids = [P.Grid.from_case(C, c) for c in cases]
    big = max(g.footprint() for g in grids)
    P.batch_reserve(C, 2 * big + 4096)
    P.batch_configure(C, graph_iters=2)  # short graphs: later solves join mid-flight
    try:
        _, first = submit_all(C, cases[:3], grids[:3])
        P.batch_run(C, 3)
        _, second = submit_all(C, cases[3:], grids[3:])
        P.batch_run(C, 2)
        _, third = submit_all(C, cases[:2], grids[:2])  # the same solves again, mid-flight
        assert P.batch_run(C, -1) == 0
    finally:
        P.batch_configure(C)
    res = collect(C, first + second + third)
    alone = [run_alone(C, c)[0] for c in cases]
    for k, (q, st, rc) in enumerate(res):
        ref = alone[k] if k < len(cases) else alone[k - len(cases)]
        assert rc == P.OK
        assert np.array_equal(q, ref), k


def test_poisoned_request_is_isolated(C):
    import paper_1711_09272_amd as P
    cases = family()[:4]
    bad = workloads.bump_case(40, np.random.Generator(np.random.PCG64(7)), 6)
    bad.q0 = bad.q0.copy()
    bad.q0[3, 5, 5] = -1.0  # negative energy: p < 0
    P.batch_reserve(C, 128 << 20)
    _, solves = submit_all(C, cases + [bad])
    P.batch_run(C, -1)
    res = collect(C, solves)
    assert res[-1][2] == P.ENONPHYS and res[-1][1]["nonphys"]
    for c, (q, st, rc) in zip(cases, res[:-1]):
        assert rc == P.OK and np.array_equal(q, run_alone(C, c)[0])


def test_batch_errors(C):
    import paper_1711_09272_amd as P
    case = workloads.bump_case(64, np.random.Generator(np.random.PCG64(1)), 3)
    g = P.Grid.from_case(C, case)
    P.batch_reserve(C, g.footprint() // 2)
    with pytest.raises(P.RoeamError) as e:
        P.batch_submit(C, [P.Solve(g, case.params, P.padded(g, case.q0), 3)])
    assert e.value.code == P.ENOMEM
    P.batch_reserve(C, 16 << 20)
    bad = dict(case.params)
    bad["cfl"] = -1.0
    with pytest.raises(P.RoeamError):
        P.batch_submit(C, [P.Solve(g, bad, P.padded(g, case.q0), 3)])
    with pytest.raises(P.RoeamError) as e:
        P.batch_poll(C, 999999)
    assert e.value.code == P.ENOTFOUND


def test_server_staggered_requests(C):
    """The request server: requests with device-built initial states submitted
    while earlier ones run each finish with the result of the same solve run
    alone, with completion times recorded."""
    import torch
    import paper_1711_09272_amd as P
    from paper_1711_09272_amd.serving import Server
    trace = workloads.serving_trace(50.0, 0.2, n_lo=24, n_hi=96, s_lo=3, s_hi=30)
    assert len(trace) >= 4
    srv = Server(C, 256 << 20)
    grids, reqs, refs = {}, [], []
    for k, tr in enumerate(trace):
        n = tr["n"]
        if n not in grids:
            grids[n] = P.Grid(C, n, n, dx=1.0 / n, dy=1.0 / n, bc=(PERIODIC,) * 4)
            grids[n].set_tile_shape(0)
        g = grids[n]
        prm = workloads.bump_params(tr["spec"]["mach"])
        q0 = workloads.bump_state_device(n, tr["spec"], g.pitch)
        q_ref = q0.clone()
        reqs.append(srv.submit(g, prm, q0, tr["steps"], tag=k))
        refs.append((g, prm, q_ref, tr["steps"]))
        if k % 2 == 1:
            srv.pump(2)
    srv.drain()
    assert not srv.outstanding and len(srv.done) == len(reqs)
    for r, (g, prm, q, n) in zip(reqs, refs):
        assert r.code == P.OK and r.stats["steps"] == n and r.latency >= 0.0
        P.step(C, g, prm, q, n)
        torch.cuda.synchronize()
        assert torch.equal(r.solve.q_out[:, :, : g.nx], q[:, :, : g.nx]), r.tag


def test_batch_profile_run_matches_batch_run(C):
    """The profiling driver runs the same kernels: bitwise the same results, one
    timed launch per stage per group per iteration, positive mean durations."""
    import paper_1711_09272_amd as P
    rng = np.random.Generator(np.random.PCG64(workloads.SEED_BASE + 51))
    cases = [workloads.bump_case(n, rng, 6) for n in (48, 70)]
    P.batch_reserve(C, 64 << 20)
    _, a = submit_all(C, cases)
    P.batch_run(C, -1)
    ra = collect(C, a)
    _, b = submit_all(C, cases)
    stage_ms, launches = P.batch_profile_run(C, -1)
    rb = collect(C, b)
    assert launches == 3 * 6 and all(t > 0.0 for t in stage_ms[:3]) and stage_ms[3] == 0.0, (stage_ms, launches)
    for (qa, sa, ca), (qb, sb, cb) in zip(ra, rb):
        assert ca == cb == P.OK and sa == sb and np.array_equal(qa, qb)


def test_graph_survives_admissions_and_retirements(C):
    """The work lists live in device memory and the graph's launches are sized
    to their capacity: after the first capture, solves admitted and retired
    within that capacity run from the same graph instance (capture counter
    unchanged), and every result is bitwise the solve run alone."""
    import paper_1711_09272_amd as P
    rng = np.random.Generator(np.random.PCG64(workloads.SEED_BASE + 52))
    waves = [[workloads.bump_case(n, rng, s) for n, s in ((64, 20), (48, 9), (80, 31))],
             [workloads.bump_case(n, rng, s) for n, s in ((56, 12), (40, 25))],
             [workloads.bump_case(n, rng, s) for n, s in ((72, 7), (64, 18), (32, 40))]]
    P.batch_reserve(C, 256 << 20)
    P.batch_configure(C, graph_iters=4)
    try:
        _, first = submit_all(C, waves[0])
        P.batch_run(C, 4)
        info0 = P.batch_info(C)
        assert info0["captures"] == 1 and info0["resident"] == 3, info0
        solves = list(first)
        for w in waves[1:]:
            _, more = submit_all(C, w)
            solves += more
            P.batch_run(C, 8)
        assert P.batch_run(C, -1) == 0
        info = P.batch_info(C)
    finally:
        P.batch_configure(C)
    say(f"[graph reuse] {info}")
    assert info["captures"] == 1 and info["graph_launches"] >= 10, info
    cases = [c for w in waves for c in w]
    for c, (q, st, rc) in zip(cases, collect(C, solves)):
        qa, sta = run_alone(C, c)
        assert rc == P.OK and st["steps"] == c.nsteps == sta["steps"]
        assert np.array_equal(q, qa), c.name


@pytest.mark.parametrize("tune", [True, False])
def test_persistent_kernels_equal_windowed(C, tune):
    """The persistent batched kernels (resident workgroups taking tiles in
    turn) give bitwise the results of one workgroup per tile, with or without
    the batch tile-shape tuning."""
    import paper_1711_09272_amd as P
    cases = family()
    out = {}
    for persistent in (False, True):
        P.batch_reserve(C, 256 << 20)
        P.batch_configure(C, persistent=persistent, autotune=tune)
        try:
            _, solves = submit_all(C, cases)
            assert P.batch_run(C, -1) == 0
            assert P.batch_info(C)["persistent"] == int(persistent)
        finally:
            P.batch_configure(C)
        out[persistent] = collect(C, solves)
    for c, (qa, sa, ca), (qb, sb, cb) in zip(cases, out[False], out[True]):
        assert ca == cb == P.OK and sa == sb and np.array_equal(qa, qb), c.name


def test_shortest_first_admission(C):
    """With room for one solve at a time, ROEAM_ADMIT_SHORTEST admits the
    queued solve of least work (cells x steps) first, FIFO the first
    submitted; results are bitwise the solves run alone either way."""
    import paper_1711_09272_amd as P
    rng = np.random.Generator(np.random.PCG64(workloads.SEED_BASE + 53))
    big, small = workloads.bump_case(96, rng, 30), workloads.bump_case(40, rng, 6)
    grids = [P.Grid.from_case(C, c) for c in (big, small)]
    for policy, first_done in ((P.ADMIT_FIFO, 0), (P.ADMIT_SHORTEST, 1)):
        P.batch_reserve(C, grids[0].footprint() + 4096)
        P.batch_configure(C, graph_iters=2, policy=policy)
        try:
            _, solves = submit_all(C, [big, small], grids)
            order = []
            while len(order) < 2:
                P.batch_run(C, 2)
                for k, s in enumerate(solves):
                    if k not in order and P.batch_poll(C, s.ticket)[0]:
                        order.append(k)
        finally:
            P.batch_configure(C)
        assert order[0] == first_done, (policy, order)
        for k, c in enumerate((big, small)):
            assert np.array_equal(solves[k].q_out[:, :, : c.nx], run_alone(C, c)[0])


@pytest.mark.parametrize("nsteps", [7, 8])
def test_forward_euler_odd_and_even_step_counts(C, nsteps):
    """Forward Euler alternates q -> qa and qa -> q with no copy between steps:
    after an odd or an even number of steps the result (single grid and
    batched) is the oracle's."""
    import paper_1711_09272_amd as P
    case = workloads.sod(nx=100, ny=3)
    case.nsteps, case.t_end = nsteps, 0.0
    q_or, st_or = oracle.run(case)
    qa, sta = run_alone(C, case)
    assert sta["steps"] == nsteps and state_error(qa, q_or) <= 1e-13
    P.batch_reserve(C, 16 << 20)
    _, solves = submit_all(C, [case])
    assert P.batch_run(C, -1) == 0
    (q, st, rc), = collect(C, solves)
    assert rc == P.OK and st["steps"] == nsteps and np.array_equal(q, qa)


def test_split_server_lanes(C):
    """Two engines on two streams: small requests batched together, large
    ones one at a time beside them, each lane pumped by its own host thread;
    every result bitwise the solve run alone."""
    import torch
    import paper_1711_09272_amd as P
    from paper_1711_09272_amd.serving import SplitServer
    trace = workloads.serving_trace(100.0, 0.1, seed=workloads.SEED_BASE + 60, n_lo=24, n_hi=160, s_lo=3, s_hi=40)
    assert len(trace) >= 6
    srv = SplitServer(0, 512 << 20, split_cells=64 * 64, graph_iters=4)
    grids, reqs, refs = {}, [], []
    try:
        for k, tr in enumerate(trace):
            n = tr["n"]
            if n not in grids:
                grids[n] = P.Grid(C, n, n, dx=1.0 / n, dy=1.0 / n, bc=(PERIODIC,) * 4)
            g = grids[n]
            prm = workloads.bump_params(tr["spec"]["mach"])
            q0 = workloads.bump_state_device(n, tr["spec"], g.pitch)
            refs.append((g, prm, q0.clone(), tr["steps"]))
            reqs.append(srv.submit(g, prm, q0, tr["steps"], tag=k))
        srv.drain()
    finally:
        srv.close()
    lanes = {n * n < 64 * 64 for n in grids}
    assert lanes == {True, False}, "both lanes used"
    for r, (g, prm, q, n) in zip(reqs, refs):
        assert r.code == P.OK and r.stats["steps"] == n, r.tag
        P.step(C, g, prm, q, n)
        torch.cuda.synchronize()
        assert torch.equal(r.solve.q_out[:, :, : g.nx], q[:, :, : g.nx]), r.tag
