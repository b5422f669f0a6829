"""Parity at the full sizes the benchmark runs, in its launch configuration:
the fourth configuration's 256 grids through the batch engine (group shape
chosen as in the bench), the 2048^2 vortex of the roofline sweep through
roeam_step with the autotuned shape, and the 128^3 extruded vortex through
roeam_step3d with the default persistent bricks (with two transported scalars:
the fallback bricks).  The oracle computes a sample of grids (always including
the largest) or the whole grid for a few steps."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import ctx, say, state_error
from workloads import PERIODIC

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    return ctx()


@pytest.mark.parametrize("precision,tol", [(1, 1e-6), (0, 1e-12)])
def test_batch256_full_size_sampled(C, precision, tol):
    import torch
    import paper_1711_09272_amd as P
    steps = 3
    cases = workloads.batch_family(256, nsteps=steps, precision=precision)
    grids = [P.Grid.from_case(C, c) for c in cases]
    q0 = [g.to_device(c.q0) for g, c in zip(grids, cases)]
    outs = [g.empty_state() for g in grids]
    P.batch_reserve(C, sum(g.footprint() for g in grids) + (64 << 20))
    solves = [P.Solve(g, c.params, q, steps, 0.0, o) for g, c, q, o in zip(grids, cases, q0, outs)]
    P.batch_submit(C, solves)
    assert P.batch_run(C, -1) == 0
    for s in solves:
        done, st, rc = P.batch_poll(C, s.ticket)
        assert done and rc == P.OK and st["steps"] == steps
    torch.cuda.synchronize()
    sizes = np.array([c.nx * c.ny for c in cases])
    rng = np.random.Generator(np.random.PCG64(workloads.SEED_BASE + 60))
    pick = sorted(set([int(sizes.argmax()), int(sizes.argmin())] + list(rng.choice(len(cases), 4, replace=False))))
    for k in pick:
        c = cases[k]
        q_or, st_or = oracle.run(c, nsteps=steps, params=dict(c.params, precision=0))
        err = state_error(grids[k].from_device(outs[k]), q_or)
        say(f"[batch256 precision {precision}] grid {k} {c.nx}x{c.ny} M={c.params['u_ref']:.3g} err {err:.3e}")
        assert err <= tol


def test_vortex2048_full_size(C):
    import paper_1711_09272_amd as P
    import torch
    case = workloads.vortex(2048, 0.01)
    g = P.Grid.from_case(C, case)
    q = g.to_device(case.q0)
    st = P.step(C, g, case.params, q, 2)
    torch.cuda.synchronize()
    q_or, st_or = oracle.run(case, nsteps=2)
    err = state_error(g.from_device(q), q_or)
    say(f"[vortex 2048^2] shape {P.SHAPES[g.tile_shape(case.params)]} 2 steps err {err:.3e}")
    assert st["steps"] == 2 and abs(st["t"] - st_or["t"]) <= 1e-13 * st_or["t"]
    assert err <= 1e-12


@pytest.mark.parametrize("precision,nsc,tol", [(0, 0, 1e-12), (1, 0, 1e-6), (0, 2, 1e-12)])
def test_vortex3d128_full_size(C, precision, nsc, tol):
    """128^3, MUSCL + SSP-RK3, two steps in the 3-D bench's launch configuration
    (default brick shape), against the FP64 oracle."""
    import paper_1711_09272_amd as P
    import torch
    case = workloads.vortex3(128, 128, 0.01, precision=precision)
    if nsc:
        case = workloads.add_scalars(case, nsc, seed=61, mode="smooth")
    g = P.Grid3.from_case(C, case)
    q = g.to_device(case.q0)
    st = P.step3(C, g, case.params, q, 2, 0.0, 0.0)
    torch.cuda.synchronize()
    q_or, st_or = oracle.run3(case, nsteps=2, params=dict(case.params, precision=0))
    err = state_error(g.from_device(q), q_or)
    say(f"[vortex3d 128^3] precision {precision}, {nsc} scalars, 2 steps err {err:.3e}")
    assert st["steps"] == 2 and abs(st["t"] - st_or["t"]) <= 1e-13 * st_or["t"]
    assert err <= tol


@pytest.mark.parametrize("reps", [3, 424])
def test_largest_grids_periodic_tiling(C, reps):
    """Near the largest grid the library accepts (nx ny < 2^31): the periodic
    64^2 vortex tiled reps x reps times (424: 27136^2 = 736 M cells, where the
    offset of the last state row, 3 x 736 M, passes 2^31 elements) is a
    periodic grid whose every cell sees the neighbourhood it has on the 64^2
    grid.  Its residual and its state after two SSP-RK3 steps (same dt: the
    max rate is the same) equal the 64^2 grid's, tiled, bit for bit.  Built and
    compared on the device, one band of 64 rows at a time."""
    import torch
    import paper_1711_09272_amd as P
    case = workloads.vortex(64, 0.01)
    n = 64 * reps
    small = P.Grid.from_case(C, case)
    qs = small.to_device(case.q0)
    r_small = P.residual(C, small, case.params, qs)[:, :, :64]
    P.step(C, small, case.params, qs, 2)
    torch.cuda.synchronize()
    q_small = qs[:, :, :64]
    big = P.Grid(C, n, n, dx=case.dx, dy=case.dy, bc=(PERIODIC,) * 4)
    say(f"[periodic tiling] {n}^2 = {n * n} cells, pitch {big.pitch}")
    q = big.empty_state()
    band = small.to_device(case.q0)[:, :, :64].repeat(1, 1, reps)
    for jb in range(reps):
        q[:, jb * 64:(jb + 1) * 64, :n] = band
    r = P.residual(C, big, case.params, q)
    r_band = r_small.repeat(1, 1, reps)
    for jb in range(reps):
        assert torch.equal(r[:, jb * 64:(jb + 1) * 64, :n], r_band), ("residual", jb)
    del r
    st = P.step(C, big, case.params, q, 2)
    torch.cuda.synchronize()
    assert st["steps"] == 2
    q_band = q_small.repeat(1, 1, reps)
    for jb in range(reps):
        assert torch.equal(q[:, jb * 64:(jb + 1) * 64, :n], q_band), ("state", jb)
    say(f"    residual and two steps equal the 64^2 grid's, tiled; t = {st['t']:.6e}")


@pytest.mark.parametrize("rxy,rz", [(2, 2), (13, 52)])
def test_largest_grids_periodic_tiling_3d(C, rxy, rz):
    """The 3-D form: the periodic 64 x 64 x 16 vortex tiled rxy x rxy x rz
    times (13, 52: 832^3 = 576 M cells, where the offset of the last state
    row, 4 x 576 M, passes 2^31 elements), through the default persistent
    bricks.  Residual and two SSP-RK3 steps equal the small grid's, tiled, bit
    for bit."""
    import torch
    import paper_1711_09272_amd as P
    case = workloads.vortex3(64, 16, 0.01)
    assert case.bc == (PERIODIC,) * 6
    nxy, nz = 64 * rxy, 16 * rz
    small = P.Grid3.from_case(C, case)
    qs = small.to_device(case.q0)
    r_small = P.residual3(C, small, case.params, qs)[..., :64]
    P.step3(C, small, case.params, qs, 2, 0.0, 0.0)
    torch.cuda.synchronize()
    q_small = qs[..., :64]
    big = P.Grid3(C, nxy, nxy, nz, case.dx, case.dy, case.dz, bc=(PERIODIC,) * 6)
    say(f"[periodic tiling 3-D] {nxy}x{nxy}x{nz} = {nxy * nxy * nz} cells, pitch {big.pitch}")
    q = big.empty_state()
    band = small.to_device(case.q0)[..., :64].repeat(1, 1, 1, rxy)
    for lb in range(rz):
        for jb in range(rxy):
            q[:, lb * 16:(lb + 1) * 16, jb * 64:(jb + 1) * 64, :nxy] = band
    r = P.residual3(C, big, case.params, q)
    r_band = r_small.repeat(1, 1, 1, rxy)
    for lb in range(rz):
        for jb in range(rxy):
            assert torch.equal(r[:, lb * 16:(lb + 1) * 16, jb * 64:(jb + 1) * 64, :nxy], r_band), ("residual", lb, jb)
    del r
    st = P.step3(C, big, case.params, q, 2, 0.0, 0.0)
    torch.cuda.synchronize()
    assert st["steps"] == 2
    q_band = q_small.repeat(1, 1, 1, rxy)
    for lb in range(rz):
        for jb in range(rxy):
            assert torch.equal(q[:, lb * 16:(lb + 1) * 16, jb * 64:(jb + 1) * 64, :nxy], q_band), ("state", lb, jb)
    say(f"    residual and two steps equal the 64x64x16 grid's, tiled; t = {st['t']:.6e}")
