"""GPU parity of the transported-scalar rows (the rho k rows of Eq. 85) on 2-D grids.

Same bars as the flow rows: FP64 residual within 1e-12 of the cancellation-aware
flux scale, FP32 coefficients within 1e-5, states after n steps within 1e-12.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import ctx, say
from workloads import DIRICHLET, PERIODIC, SLIPWALL, TRANSMISSIVE

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def C():
    return ctx()


def rerr(r, r_or, sc):
    return np.array([np.abs(r[k] - r_or[k]).max() / sc[k].max() for k in range(r.shape[0])])


def gpu_residual(c, case, params=None, shape=None):
    import torch
    import paper_1711_09272_amd as P
    g = P.Grid.from_case(c, case)
    if shape is not None:
        g.set_tile_shape(shape)
    r = P.residual(c, g, params or case.params, g.to_device(case.q0))
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


def cases():
    yield "smooth_periodic_1", workloads.add_scalars(
        workloads.smooth_random_case(75, 37, 1, order=2, eps1=1.0, mach_ref=0.05), 1, seed=1)
    yield "smooth_nodes_walls_2", workloads.add_scalars(
        workloads.smooth_random_case(45, 29, 2, bc=(DIRICHLET, TRANSMISSIVE, SLIPWALL, SLIPWALL), nodes=True, order=2,
                                     eps1=1.0), 2, seed=2, k_bc=np.array([[0.5, 1.5]] * 4))
    yield "order1_bcmix_2", workloads.add_scalars(
        workloads.smooth_random_case(33, 16, 3, bc=(TRANSMISSIVE, DIRICHLET, PERIODIC, PERIODIC), order=1), 2, seed=3,
        mode="smooth")
    yield "classical_roe_1", workloads.add_scalars(workloads.smooth_random_case(40, 20, 4, order=2, scheme=1), 1,
                                                   seed=4)
    yield "roe_harten_walls_2", workloads.add_scalars(
        workloads.smooth_random_case(40, 20, 5, bc=(SLIPWALL, DIRICHLET, TRANSMISSIVE, SLIPWALL), order=2, scheme=2,
                                     eps_lambda=0.2), 2, seed=5)
    yield "ablations_1", workloads.add_scalars(
        workloads.smooth_random_case(33, 16, 6, order=2, eps1=1.0, variant=2 | 4 | 64 | 128), 1, seed=6)
    yield "s1_one_2", workloads.add_scalars(workloads.smooth_random_case(33, 16, 7, order=2, eps1=1.0, s1_mode=1), 2,
                                            seed=7)
    yield "min_2x2_2", workloads.add_scalars(workloads.smooth_random_case(2, 2, 8, order=2, eps1=1.0), 2, seed=8)
    yield "vortex_256_1", workloads.add_scalars(workloads.vortex(256, 0.01), 1, seed=9, mode="smooth")


CASES = list(cases())


@pytest.mark.parametrize("name,case", CASES, ids=[n for n, _ in CASES])
def test_residual_with_scalars_fp64(C, name, case):
    say(f"[scalars residual fp64] {name} {case.nx}x{case.ny} ns={case.nscalars}")
    r_or, sc = oracle.residual(case, with_scale=True)
    r = gpu_residual(C, case)
    err = rerr(r, r_or, sc)
    say(f"    err per row {err}")
    assert np.all(err <= TOL64), err


@pytest.mark.parametrize("name", ["smooth_periodic_1", "smooth_nodes_walls_2", "vortex_256_1"])
def test_residual_with_scalars_fp32_flux(C, name):
    case = dict(CASES)[name]
    r_or, sc = oracle.residual(case, with_scale=True)
    r = gpu_residual(C, case, params=dict(case.params, precision=1))
    err = rerr(r, r_or, sc)
    say(f"[scalars residual fp32] {name} err {err}")
    assert np.all(err <= TOL32), err


def test_flow_rows_do_not_see_the_scalars(C):
    base = workloads.smooth_random_case(45, 29, 10, bc=(DIRICHLET, TRANSMISSIVE, SLIPWALL, SLIPWALL), nodes=True,
                                       order=2, eps1=1.0)
    r0 = gpu_residual(C, base)
    _, sc = oracle.residual(base, with_scale=True)
    for ns in (1, 2):
        r = gpu_residual(C, workloads.add_scalars(base, ns, seed=ns))
        say(f"[flow rows, {ns} scalars] bitwise equal: {np.array_equal(r[:4], r0)}")
        assert np.all(rerr(r[:4], r0, sc) <= 1e-14)


def test_unit_scalar_follows_the_mass_row(C):
    base = workloads.smooth_random_case(40, 20, 11, bc=(DIRICHLET, TRANSMISSIVE, SLIPWALL, SLIPWALL), order=2,
                                        eps1=1.0)
    c = workloads.add_scalars(base, 1, mode="const", value=1.0)
    r = gpu_residual(C, c)
    _, sc = oracle.residual(c, with_scale=True)
    assert np.abs(r[4] - r[0]).max() <= 1e-14 * sc[0].max()


@pytest.mark.parametrize("shape", range(9))
def test_every_tile_shape_with_scalars(C, shape):
    case = dict(CASES)["smooth_nodes_walls_2"]
    r0 = gpu_residual(C, case, shape=6)
    r = gpu_residual(C, case, shape=shape)
    assert np.array_equal(r, r0)


@pytest.mark.parametrize("ts,steps", [(0, 6), (1, 5), (2, 4)])
def test_steps_with_scalars(C, ts, steps):
    base = workloads.smooth_random_case(45, 29, 12, bc=(DIRICHLET, TRANSMISSIVE, SLIPWALL, SLIPWALL), nodes=True,
                                        order=2, eps1=1.0, time_scheme=ts)
    case = workloads.add_scalars(base, 2, seed=12, k_bc=np.array([[0.5, 1.5]] * 4))
    say(f"[scalars steps] time scheme {ts}, {steps} steps")
    q_or, st_or = oracle.run(case, nsteps=steps)
    q, st = gpu_run(C, case, steps)
    err = np.abs(q - q_or).max() / np.abs(q_or).max()
    say(f"    err {err:.3e}")
    assert st["steps"] == steps and abs(st["t"] - st_or["t"]) <= 1e-13 * st_or["t"]
    assert err <= TOL64


def test_vortex_with_scalar_steps(C):
    case = workloads.add_scalars(workloads.vortex(128, 0.01), 1, seed=13, mode="smooth")
    q_or, _ = oracle.run(case, nsteps=10)
    q, st = gpu_run(C, case, 10)
    assert st["steps"] == 10 and np.abs(q - q_or).max() / np.abs(q_or).max() <= TOL64


def test_scalar_arguments(C):
    import paper_1711_09272_amd as P
    base = workloads.smooth_random_case(16, 8, 14, bc=(DIRICHLET, TRANSMISSIVE, PERIODIC, PERIODIC))
    g = P.Grid.from_case(C, base)
    with pytest.raises(P.RoeamError):
        g.set_scalars(3)
    with pytest.raises(P.RoeamError):
        g.set_scalars(1)  # Dirichlet side without scalars
    g.set_scalars(1, np.ones((4, 1)))
    assert g.empty_state().shape[0] == 5
    g.set_scalars(0)
    assert g.empty_state().shape[0] == 4
    g.set_scalars(2, np.ones((4, 2)))
    assert g.empty_state().shape[0] == 6
