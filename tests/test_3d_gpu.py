"""GPU parity of the 3-D path (uniform Cartesian grids) against the 3-D FP64 oracle.

Same bar as the 2-D parity tests: FP64 residual within 1e-12 of the
cancellation-aware scale (max over cells of sum_faces |F_k| A / V), FP32-flux
residual within 1e-5, states after n steps within 1e-12 of max |Q|.  Grids span
several bricks of every shape with ragged tails in all three directions.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import ctx, say
from paper_1711_09272_amd import SHAPES3
from workloads import DIRICHLET, PERIODIC, SLIPWALL, TRANSMISSIVE

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def C():
    return ctx()


def gpu_residual3(c, case, params=None, shape=None):
    import torch
    import paper_1711_09272_amd as P
    g = P.Grid3.from_case(c, case)
    if shape is not None:
        g.set_tile_shape(shape)
    q = g.to_device(case.q0)
    rate_t = torch.zeros(1, dtype=torch.float64, device="cuda")
    r = P.residual3(c, g, params or case.params, q, rate_out=rate_t)
    torch.cuda.synchronize()
    return g.from_device(r), float(rate_t.item())


def gpu_run3(c, case, nsteps, t_end=0.0, params=None, shape=None, q0=None):
    import torch
    import paper_1711_09272_amd as P
    g = P.Grid3.from_case(c, case)
    if shape is not None:
        g.set_tile_shape(shape)
    q = g.to_device(case.q0 if q0 is None else q0)
    st = P.step3(c, g, params or case.params, q, nsteps, 0.0, t_end)
    torch.cuda.synchronize()
    return g.from_device(q), st


def rerr(r, r_or, scale):
    return np.array([np.abs(r[k] - r_or[k]).max() / scale[k].max() for k in range(5)])


def serr(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


ALL_WALLS = (TRANSMISSIVE, DIRICHLET, SLIPWALL, SLIPWALL, DIRICHLET, SLIPWALL)


def residual_cases():
    yield "smooth_periodic_19x13x11", workloads.smooth_random_case3(19, 13, 11, 1, order=2, eps1=1.0, mach_ref=0.05)
    yield "smooth_walls_18x11x10", workloads.smooth_random_case3(18, 11, 10, 2, bc=ALL_WALLS, order=2, eps1=1.0)
    yield "smooth_walls2_order1", workloads.smooth_random_case3(
        17, 9, 6, 3, bc=(DIRICHLET, TRANSMISSIVE, TRANSMISSIVE, SLIPWALL, SLIPWALL, TRANSMISSIVE), order=1, eps1=0.0)
    yield "rough_periodic_21x10x9", workloads.rough_case3(21, 10, 9, 4, order=2, eps1=1.0, mach_ref=0.01)
    yield "rough_walls_order1", workloads.rough_case3(13, 9, 7, 5, bc=ALL_WALLS, order=1, eps1=1.0)
    yield "rough_s1_one", workloads.rough_case3(12, 9, 6, 6, order=2, eps1=1.0, s1_mode=1)
    yield "rough_xi_ungated", workloads.rough_case3(12, 9, 6, 7, order=2, eps1=1.0, variant=1)
    yield "rough_expfix_f8_clamp", workloads.rough_case3(12, 9, 6, 8, order=2, eps1=1.0, variant=2 | 4)
    yield "rough_ablation_noeq92_xiroe_duproe", workloads.rough_case3(12, 9, 6, 9, order=2, eps1=1.0, variant=8 | 16 | 32)
    yield "rough_ablation_xieq46_dupzero", workloads.rough_case3(12, 9, 6, 10, order=2, eps1=1.0, variant=64 | 128)
    yield "rough_classical_roe", workloads.rough_case3(12, 9, 6, 11, order=2, scheme=1)
    yield "rough_roe_harten", workloads.rough_case3(12, 9, 6, 12, order=2, scheme=2, eps_lambda=0.2)
    yield "min_2x2x2_periodic", workloads.smooth_random_case3(2, 2, 2, 13, order=2, eps1=1.0)
    yield "min_2x3x2_walls", workloads.smooth_random_case3(2, 3, 2, 14, bc=ALL_WALLS, order=2)
    yield "vortex3_64x64x16", workloads.vortex3(64, 16, 0.01)


CASES = list(residual_cases())


@pytest.mark.parametrize("name,case", CASES, ids=[n for n, _ in CASES])
def test_residual3_fp64(C, name, case):
    say(f"[residual3 fp64] {name} {case.nx}x{case.ny}x{case.nz}")
    r_or, scale = oracle.residual3(case, with_scale=True)
    r, rate = gpu_residual3(C, case)
    err = rerr(r, r_or, scale)
    say(f"    err per row {err}")
    assert np.all(err <= TOL64), err
    rate_or = oracle.max_rate3(case)
    assert abs(rate - rate_or) <= 1e-14 * rate_or


@pytest.mark.parametrize("name", ["smooth_periodic_19x13x11", "rough_periodic_21x10x9", "vortex3_64x64x16"])
def test_residual3_fp32_flux(C, name):
    case = dict(CASES)[name]
    say(f"[residual3 fp32-flux] {name}")
    r_or, scale = oracle.residual3(case, with_scale=True)
    prm = dict(case.params, precision=1)
    r, _ = gpu_residual3(C, case, params=prm)
    err = rerr(r, r_or, scale)
    say(f"    err per row {err}")
    assert np.all(err <= TOL32), err


# the z-marching shapes (column tiles walking runs of planes)
ZSHAPES = [k for k, name in enumerate(SHAPES3) if "z" in name]


@pytest.mark.parametrize("shape", range(len(SHAPES3)))
def test_every_brick_shape_is_bitwise_identical(C, shape):
    """All brick shapes evaluate the same faces with the same arithmetic."""
    case = workloads.rough_case3(37, 19, 13, 15, bc=ALL_WALLS, order=2, eps1=1.0, mach_ref=0.05)
    say(f"[brick shape {shape}] 37x19x13")
    r0, _ = gpu_residual3(C, case, shape=0)
    r, _ = gpu_residual3(C, case, shape=shape)
    assert np.array_equal(r, r0)
    r_or, scale = oracle.residual3(case, with_scale=True)
    assert np.all(rerr(r, r_or, scale) <= TOL64)


@pytest.mark.parametrize("name,case", CASES, ids=[n for n, _ in CASES])
@pytest.mark.parametrize("shape", [ZSHAPES[0], ZSHAPES[-1]])
def test_zmarch_residual_every_case(C, shape, name, case):
    """The z-marching kernel on every residual case (boundary kinds, orders,
    schemes, variants, the 2-cell grids): bitwise the brick kernel's result,
    rate included."""
    say(f"[z-march shape {shape}] {name} {case.nx}x{case.ny}x{case.nz}")
    r0, rate0 = gpu_residual3(C, case, shape=0)
    r, rate = gpu_residual3(C, case, shape=shape)
    assert np.array_equal(r, r0) and rate == rate0


@pytest.mark.parametrize("shape", [8, 9] + ZSHAPES)
@pytest.mark.parametrize("ts,steps", [(0, 3), (1, 2), (2, 2)])
def test_persistent_bricks_steps(C, shape, ts, steps):
    """The persistent and z-marching shapes on a grid with more bricks or runs
    than resident workgroups (64^3: 512 bricks; 20 column tiles x 16, 8 or 4
    runs): every stage code, the step state and the rate reduction, bitwise
    equal to the one-brick-per-workgroup kernel and within 1e-12 of the
    oracle."""
    case = workloads.smooth_random_case3(64, 64, 64, 30, bc=ALL_WALLS, order=2, eps1=1.0, mach_ref=0.05,
                                         time_scheme=ts, cfl=0.4)
    say(f"[persistent shape {shape}] time scheme {ts}, {steps} steps, 64^3")
    q6, st6 = gpu_run3(C, case, steps, shape=6)
    q, st = gpu_run3(C, case, steps, shape=shape)
    assert st["steps"] == steps and st["t"] == st6["t"]
    assert np.array_equal(q, q6)
    q_or, st_or = oracle.run3(case, nsteps=steps)
    say(f"    err {serr(q, q_or):.3e}")
    assert serr(q, q_or) <= TOL64 and abs(st["t"] - st_or["t"]) <= 1e-13 * st_or["t"]
    r6, rate6 = gpu_residual3(C, case, shape=6)
    r, rate = gpu_residual3(C, case, shape=shape)
    assert np.array_equal(r, r6) and rate == rate6


def test_default_shape_follows_the_grid_size(C):
    """By default a 3-D grid runs the z-marching shape with the longest run
    whose workgroups number at least nine per CU (three rounds of the three a
    CU holds), else the shortest run; a set shape is kept."""
    import torch
    import paper_1711_09272_amd as P
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    runs = {k: int(name.split("z")[1].split("/")[0]) for k, name in enumerate(SHAPES3) if "z" in name and "*" not in name}

    def expected(n, nz):
        tiles = -(-n // 16) * -(-n // 15)
        fit = [k for k, zc in runs.items() if tiles * -(-nz // zc) >= 9 * cus]
        return max(fit, key=runs.get) if fit else min(runs, key=runs.get)

    for n, nz in ((32, 8), (128, 128), (256, 256), (512, 64)):
        g = P.Grid3(C, n, n, nz, 0.1, 0.1, 0.1)
        assert g.tile_shape(2) == expected(n, nz), (n, nz, g.tile_shape(2))
        g.set_tile_shape(8)
        assert g.tile_shape(2) == 8
        g.close()
    say(f"[default 3-D shape] {cus} CUs: 128^3 -> {SHAPES3[expected(128, 128)]}, 256^3 -> {SHAPES3[expected(256, 256)]}")


def test_extruded_2d_case_matches_the_2d_oracle(C):
    """A 2-D case repeated along a periodic z: every z-slice of the 3-D GPU
    residual is the 2-D oracle residual and the w row is zero."""
    c2 = workloads.smooth_random_case(23, 14, 16, bc=(TRANSMISSIVE, DIRICHLET, SLIPWALL, SLIPWALL), order=2,
                                      eps1=1.0, mach_ref=0.05)
    c3 = workloads.extrude(c2, 5)
    c3.dz = 0.37
    say("[extruded] 23x14 x 5")
    r2, sc2 = oracle.residual(c2, with_scale=True)
    r3, _ = gpu_residual3(C, c3)
    for l in range(5):
        for k2, k3 in ((0, 0), (1, 1), (2, 2), (3, 4)):
            assert np.abs(r3[k3, l] - r2[k2]).max() <= TOL64 * sc2[k2].max()
    assert np.abs(r3[3]).max() == 0.0


@pytest.mark.parametrize("ts,steps", [(0, 4), (1, 3), (2, 3)])
def test_steps3_match_oracle(C, ts, steps):
    case = workloads.smooth_random_case3(19, 13, 11, 16, bc=ALL_WALLS, order=2, eps1=1.0, mach_ref=0.05,
                                         time_scheme=ts, cfl=0.4)
    say(f"[step3] time scheme {ts}, {steps} steps, 19x13x11")
    q_or, st_or = oracle.run3(case, nsteps=steps)
    q, st = gpu_run3(C, case, steps)
    say(f"    err {serr(q, q_or):.3e} t {st['t']:.6e} (oracle {st_or['t']:.6e})")
    assert st["steps"] == steps
    assert abs(st["t"] - st_or["t"]) <= 1e-13 * st_or["t"]
    assert serr(q, q_or) <= TOL64


def test_vortex3_steps(C):
    case = workloads.vortex3(64, 16, 0.01, time_scheme=1)
    say("[step3] vortex3 64x64x16 M=0.01, 8 SSP-RK3 steps")
    q_or, st_or = oracle.run3(case, nsteps=8)
    q, st = gpu_run3(C, case, 8)
    say(f"    err {serr(q, q_or):.3e}")
    assert st["steps"] == 8 and serr(q, q_or) <= TOL64


def test_t_end_lands_exactly_3d(C):
    case = workloads.smooth_random_case3(10, 9, 8, 17, order=1, time_scheme=0)
    rate = oracle.max_rate3(case)
    t_end = 2.5 * case.params["cfl"] / rate
    q_or, st_or = oracle.run3(case, nsteps=1000, t_end=t_end)
    q, st = gpu_run3(C, case, 1000, t_end=t_end)
    assert st["t"] == t_end and st["steps"] == st_or["steps"]
    assert serr(q, q_or) <= TOL64


def test_nonphysical_state_is_reported_3d(C):
    import paper_1711_09272_amd as P
    case = workloads.smooth_random_case3(8, 8, 8, 18, order=2)
    q0 = case.q0.copy()
    q0[4, 3, 4, 5] = 0.0  # rho E = 0: negative pressure
    with pytest.raises(P.NonPhysicalError):
        gpu_run3(C, case, 3, q0=q0)


def test_invalid_arguments_3d(C):
    import paper_1711_09272_amd as P
    with pytest.raises(P.RoeamError):
        P.Grid3(C, 1, 4, 4, 0.1, 0.1, 0.1)
    with pytest.raises(P.RoeamError):
        P.Grid3(C, 4, 4, 4, 0.1, 0.0, 0.1)
    with pytest.raises(P.RoeamError):
        P.Grid3(C, 4, 4, 4, 0.1, 0.1, 0.1, bc=(PERIODIC,) * 4 + (PERIODIC, SLIPWALL))
    with pytest.raises(P.RoeamError):
        P.Grid3(C, 4, 4, 4, 0.1, 0.1, 0.1, bc=(DIRICHLET,) + (PERIODIC,) * 5)
    case = workloads.smooth_random_case3(4, 4, 4, 19)
    g = P.Grid3.from_case(C, case)
    with pytest.raises(P.RoeamError):
        g.set_tile_shape(len(SHAPES3))
    q = g.to_device(case.q0)
    with pytest.raises(P.RoeamError):
        P.residual3(C, g, dict(case.params, order=3), q)


def test_graph_replays_match_eager_steps_3d(C):
    """The 3-D step's captured graph, replayed across calls with torch work and
    host synchronisations between them, and replayed three times within one
    call, gives the eager one-step-per-call states bit for bit."""
    import torch
    import paper_1711_09272_amd as P
    case = workloads.vortex3(24, 8, 0.01, time_scheme=1)
    g = P.Grid3.from_case(C, case)
    q = g.to_device(case.q0)
    t, snaps = 0.0, {}
    for k in range(1, 111):
        t = P.step3(C, g, case.params, q, 1, t)["t"]
        if k % 6 == 0 or k == 110:
            snaps[k] = (g.from_device(q), t)
    q2 = g.to_device(case.q0)
    t = 0.0
    for k in (6, 12, 18):
        t = P.step3(C, g, case.params, q2, 6, t)["t"]
        x = torch.randn(1 << 16, device="cuda", dtype=torch.float64)
        float((x * x).sum())
        torch.cuda.synchronize()
        assert np.array_equal(g.from_device(q2), snaps[k][0]) and t == snaps[k][1], k
    q3 = g.to_device(case.q0)
    st = P.step3(C, g, case.params, q3, 110)
    torch.cuda.synchronize()
    say(f"[graph replays 3-D] 110 steps to t = {st['t']:.6e}")
    assert st["steps"] == 110 and st["t"] == snaps[110][1]
    assert np.array_equal(g.from_device(q3), snaps[110][0])
