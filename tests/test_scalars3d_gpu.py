"""GPU parity of the transported-scalar rows (the rho k rows of Eq. 85) on 3-D grids.

Same bars as the flow rows: FP64 residual within 1e-12 of the cancellation-aware
flux scale, FP32 coefficients within 1e-5, states after n steps within 1e-12.
"""
import numpy as np
import pytest

import oracle
import workloads
from paper_1711_09272_amd import SHAPES3
from gpu_util import ctx, say
from workloads import DIRICHLET, PERIODIC, SLIPWALL, TRANSMISSIVE

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5
ALL_WALLS = (TRANSMISSIVE, DIRICHLET, SLIPWALL, SLIPWALL, DIRICHLET, SLIPWALL)


@pytest.fixture(scope="module")
def C():
    return ctx()


def rerr(r, r_or, sc):
    return np.array([np.abs(r[k] - r_or[k]).max() / sc[k].max() for k in range(r.shape[0])])


def gpu_residual3(c, case, params=None, shape=None):
    import torch
    import paper_1711_09272_amd as P
    g = P.Grid3.from_case(c, case)
    if shape is not None:
        g.set_tile_shape(shape)
    rate_t = torch.zeros(1, dtype=torch.float64, device="cuda")
    r = P.residual3(c, g, params or case.params, g.to_device(case.q0), rate_out=rate_t)
    torch.cuda.synchronize()
    return g.from_device(r), float(rate_t.item())


def gpu_run3(c, case, nsteps, t_end=0.0, shape=None):
    import torch
    import paper_1711_09272_amd as P
    g = P.Grid3.from_case(c, case)
    if shape is not None:
        g.set_tile_shape(shape)
    q = g.to_device(case.q0)
    st = P.step3(c, g, case.params, q, nsteps, 0.0, t_end)
    torch.cuda.synchronize()
    return g.from_device(q), st


def cases():
    yield "smooth_periodic_1", workloads.add_scalars(
        workloads.smooth_random_case3(19, 13, 11, 1, order=2, eps1=1.0, mach_ref=0.05), 1, seed=1)
    yield "smooth_walls_2", workloads.add_scalars(
        workloads.smooth_random_case3(18, 11, 10, 2, bc=ALL_WALLS, order=2, eps1=1.0), 2, seed=2,
        k_bc=np.array([[0.5, 1.5]] * 6))
    yield "order1_walls_2", workloads.add_scalars(
        workloads.smooth_random_case3(17, 9, 6, 3, bc=(DIRICHLET, TRANSMISSIVE, TRANSMISSIVE, SLIPWALL, SLIPWALL,
                                                       TRANSMISSIVE), order=1), 2, seed=3, mode="smooth")
    yield "rough_periodic_2", workloads.add_scalars(workloads.rough_case3(21, 10, 9, 4, order=2, eps1=1.0,
                                                                          mach_ref=0.01), 2, seed=4)
    yield "rough_classical_roe_1", workloads.add_scalars(workloads.rough_case3(12, 9, 6, 11, order=2, scheme=1), 1,
                                                         seed=5)
    yield "rough_roe_harten_walls_2", workloads.add_scalars(
        workloads.rough_case3(12, 9, 6, 12, bc=ALL_WALLS, order=2, scheme=2, eps_lambda=0.2), 2, seed=6)
    yield "rough_ablations_1", workloads.add_scalars(
        workloads.rough_case3(12, 9, 6, 10, order=2, eps1=1.0, variant=2 | 4 | 64 | 128), 1, seed=7)
    yield "rough_s1_one_2", workloads.add_scalars(workloads.rough_case3(12, 9, 6, 6, order=2, eps1=1.0, s1_mode=1), 2,
                                                  seed=8)
    yield "min_2x2x2_2", workloads.add_scalars(workloads.smooth_random_case3(2, 2, 2, 13, order=2, eps1=1.0), 2,
                                               seed=9)
    yield "vortex3_64x64x16_1", workloads.add_scalars(workloads.vortex3(64, 16, 0.01), 1, seed=10, mode="smooth")


CASES = list(cases())


@pytest.mark.parametrize("name,case", CASES, ids=[n for n, _ in CASES])
def test_residual3_with_scalars_fp64(C, name, case):
    ns = case.q0.shape[0] - 5
    say(f"[scalars3 residual fp64] {name} {case.nx}x{case.ny}x{case.nz} ns={ns}")
    r_or, sc = oracle.residual3(case, with_scale=True)
    r, rate = gpu_residual3(C, case)
    err = rerr(r, r_or, sc)
    say(f"    err per row {err}")
    assert np.all(err <= TOL64), err
    rate_or = oracle.max_rate3(case)
    assert abs(rate - rate_or) <= 1e-14 * rate_or


@pytest.mark.parametrize("name", ["smooth_periodic_1", "rough_periodic_2", "vortex3_64x64x16_1"])
def test_residual3_with_scalars_fp32_flux(C, name):
    case = dict(CASES)[name]
    r_or, sc = oracle.residual3(case, with_scale=True)
    r, _ = gpu_residual3(C, case, params=dict(case.params, precision=1))
    err = rerr(r, r_or, sc)
    say(f"[scalars3 residual fp32] {name} err {err}")
    assert np.all(err <= TOL32), err


def test_flow_rows_do_not_see_the_scalars_3d(C):
    base = workloads.rough_case3(15, 9, 7, 20, bc=ALL_WALLS, order=2, eps1=1.0)
    r0, _ = gpu_residual3(C, base)
    for ns in (1, 2):
        r, _ = gpu_residual3(C, workloads.add_scalars(base, ns, seed=ns))
        say(f"[flow rows 3-D, {ns} scalars]")
        assert np.array_equal(r[:5], r0)


def test_unit_scalar_follows_the_mass_row_3d(C):
    base = workloads.smooth_random_case3(16, 10, 9, 21, bc=ALL_WALLS, order=2, eps1=1.0)
    c = workloads.add_scalars(base, 1, mode="const", value=1.0)
    r, _ = gpu_residual3(C, c)
    _, sc = oracle.residual3(c, with_scale=True)
    assert np.abs(r[5] - r[0]).max() <= 1e-14 * sc[0].max()


@pytest.mark.parametrize("ns", [1, 2])
@pytest.mark.parametrize("shape", range(len(SHAPES3)))
def test_every_brick_shape_with_scalars(C, shape, ns):
    """Every shape computes the same bits; with two scalars the 16x8x4 bricks do
    not fit the LDS and run the fallback shape (persistent 8x8x8), again the
    same bits."""
    case = workloads.add_scalars(workloads.rough_case3(37, 19, 13, 15, bc=ALL_WALLS, order=2, eps1=1.0,
                                                       mach_ref=0.05), ns, seed=22)
    say(f"[brick shape {shape}, {ns} scalars] 37x19x13")
    r0, _ = gpu_residual3(C, case, shape=0)
    r, _ = gpu_residual3(C, case, shape=shape)
    assert np.array_equal(r, r0)


@pytest.mark.parametrize("ts,steps", [(0, 4), (1, 3), (2, 3)])
def test_steps3_with_scalars(C, ts, steps):
    base = workloads.smooth_random_case3(19, 13, 11, 16, bc=ALL_WALLS, order=2, eps1=1.0, mach_ref=0.05,
                                         time_scheme=ts, cfl=0.4)
    case = workloads.add_scalars(base, 2, seed=23, k_bc=np.array([[0.5, 1.5]] * 6))
    say(f"[scalars3 steps] time scheme {ts}, {steps} steps")
    q_or, st_or = oracle.run3(case, nsteps=steps)
    q, st = gpu_run3(C, case, steps)
    err = np.abs(q - q_or).max() / np.abs(q_or).max()
    say(f"    err {err:.3e}")
    assert st["steps"] == steps and abs(st["t"] - st_or["t"]) <= 1e-13 * st_or["t"]
    assert err <= TOL64


def test_vortex3_with_scalar_steps_default_shape(C):
    """SSP-RK3 on the extruded vortex with two scalars through the default brick
    shape (which falls back for two scalars) and with one scalar."""
    for ns in (1, 2):
        case = workloads.add_scalars(workloads.vortex3(64, 16, 0.01, time_scheme=1), ns, seed=24, mode="smooth")
        q_or, _ = oracle.run3(case, nsteps=6)
        q, st = gpu_run3(C, case, 6)
        err = np.abs(q - q_or).max() / np.abs(q_or).max()
        say(f"[vortex3 scalars] ns={ns} err {err:.3e}")
        assert st["steps"] == 6 and err <= TOL64


def test_residual_norms3_with_scalars(C):
    import torch
    import paper_1711_09272_amd as P
    case = workloads.add_scalars(workloads.smooth_random_case3(19, 13, 11, 5, order=2, eps1=1.0), 2, seed=25)
    g = P.Grid3.from_case(C, case)
    r = P.residual3(C, g, case.params, g.to_device(case.q0))
    a = P.residual_norms(C, g, r).cpu().numpy()
    torch.cuda.synchronize()
    flat = g.from_device(r).reshape(7, -1)
    assert a.shape == (2, 7)
    assert np.allclose(a[0], np.sqrt((flat * flat).mean(axis=1)), rtol=1e-13, atol=0)
    assert np.array_equal(a[1], np.abs(flat).max(axis=1))


def test_scalar_arguments_3d(C):
    import paper_1711_09272_amd as P
    base = workloads.smooth_random_case3(6, 5, 4, 26, bc=(DIRICHLET, TRANSMISSIVE) + (PERIODIC,) * 4)
    g = P.Grid3.from_case(C, base)
    with pytest.raises(P.RoeamError):
        g.set_scalars(3)
    with pytest.raises(P.RoeamError):
        g.set_scalars(1)  # Dirichlet side without scalars
    with pytest.raises(P.RoeamError):
        g.set_scalars(1, np.full((6, 1), np.nan))
    g.set_scalars(1, np.ones((6, 1)))
    assert g.empty_state().shape[0] == 6
    g.set_scalars(0)
    assert g.empty_state().shape[0] == 5
