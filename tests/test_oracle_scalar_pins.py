"""Pins of the oracle's transported-scalar rows (the rho k rows of Eq. 85).

A passive scalar rides on the mass flux: with k = 1 its row must be the mass
row, with k = c it must be c times it, and in a uniform flow the scheme reduces
to upwind advection of k (xi = |U|, dU_p = dU_u = 0), a textbook closed form.
The classical Roe row is checked against the eigen-decomposition of the Roe
matrix extended by the scalar.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from workloads import DIRICHLET, PERIODIC, SLIPWALL, TRANSMISSIVE

G = 1.4


def base_cases():
    yield workloads.smooth_random_case(23, 13, 1, order=2, eps1=1.0, mach_ref=0.05)
    yield workloads.smooth_random_case(21, 12, 2, bc=(TRANSMISSIVE, DIRICHLET, SLIPWALL, SLIPWALL), nodes=True,
                                       order=2, eps1=1.0)
    yield workloads.smooth_random_case(17, 9, 3, bc=(DIRICHLET, TRANSMISSIVE, PERIODIC, PERIODIC), order=1)
    yield workloads.smooth_random_case(15, 11, 4, order=2, scheme=1)
    yield workloads.smooth_random_case(15, 11, 5, bc=(SLIPWALL, DIRICHLET, TRANSMISSIVE, SLIPWALL), order=2,
                                       scheme=2, eps_lambda=0.2)
    yield workloads.smooth_random_case(15, 11, 6, order=2, eps1=1.0, variant=2 | 4 | 64 | 128)


CASES = list(base_cases())


@pytest.mark.parametrize("k", range(len(CASES)))
def test_unit_scalar_row_is_the_mass_row(k):
    c = workloads.add_scalars(CASES[k], 1, mode="const", value=1.0)
    r = oracle.residual(c)
    assert np.array_equal(r[4], r[0])
    assert np.array_equal(r[:4], oracle.residual(CASES[k]))  # the flow does not see the scalar


@pytest.mark.parametrize("k", range(len(CASES)))
def test_constant_scalar_scales_the_mass_row(k):
    c = workloads.add_scalars(CASES[k], 1, mode="const", value=0.3)
    r, sc = oracle.residual(c, with_scale=True)
    assert np.abs(r[4] - 0.3 * r[0]).max() <= 1e-14 * sc[0].max()


@pytest.mark.parametrize("k", range(len(CASES)))
def test_second_scalar_twice_the_first(k):
    """Both scalar slots are treated alike: k_2 = 2 k_1 gives R_2 = 2 R_1 exactly
    (scaling by two commutes with every rounding)."""
    c = workloads.add_scalars(CASES[k], 2, seed=k, mode="double")
    r = oracle.residual(c)
    assert np.array_equal(r[5], 2.0 * r[4])


def _minmod(a, b):
    return np.where(a * b <= 0.0, 0.0, np.sign(a) * np.minimum(np.abs(a), np.abs(b)))


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("mach,sx,sy,scheme", [(0.3, 1, 1, 0), (0.3, -1, 1, 0), (1.7, 1, -1, 0), (0.6, -1, -1, 1)])
def test_uniform_flow_is_upwind_advection(order, mach, sx, sy, scheme):
    """Uniform rho, V, p with a rough k: the scalar flux is U rho k of the
    upwind face state (first order: the upwind cell; MUSCL: its minmod-limited
    extrapolation), and the flow rows stay at zero."""
    nx, ny = 24, 14
    dx, dy = 0.1, 0.07
    rho, p = 1.3, 0.9
    cs = math.sqrt(G * p / rho)
    u, v = sx * mach * cs * 0.8, sy * mach * cs * 0.6
    q0 = np.zeros((4, ny, nx))
    q0[:] = workloads.conserved(G, rho, u, v, p)[:, None, None]
    base = workloads.Case(name="uniform", q0=q0, params=workloads.default_params(order=order, eps1=1.0,
                                                                                 mach_ref=0.3, u_ref=abs(u),
                                                                                 scheme=scheme, eps_lambda=0.0),
                          bc=(PERIODIC,) * 4, dx=dx, dy=dy)
    c = workloads.add_scalars(base, 1, seed=7, mode="rough")
    r, sc = oracle.residual(c, with_scale=True)
    k = c.q0[4] / c.q0[0]

    def upwind(kk, vel, axis):
        # face f between cells f-1 and f along the axis (periodic)
        km1, km2, kp0, kp1 = (np.roll(kk, s, axis=axis) for s in (1, 2, 0, -1))
        if order == 1:
            kl, kr = km1, kp0
        else:
            kl = km1 + 0.5 * _minmod(km1 - km2, kp0 - km1)
            kr = kp0 - 0.5 * _minmod(kp0 - km1, kp1 - kp0)
        return vel * rho * (kl if vel > 0 else kr)

    fx = upwind(k, u, 1) * dy
    fy = upwind(k, v, 0) * dx
    ref = -((np.roll(fx, -1, axis=1) - fx) + (np.roll(fy, -1, axis=0) - fy)) / (dx * dy)
    assert np.abs(r[4] - ref).max() <= 1e-13 * sc[4].max()
    assert np.abs(r[:4]).max() <= 1e-13 * sc[:4].max()


def test_scalar_conservation_on_a_periodic_node_grid():
    c = workloads.add_scalars(workloads.smooth_random_case(26, 15, 8, nodes=True, order=2, eps1=1.0), 2, seed=3)
    r, sc = oracle.residual(c, with_scale=True)
    om = oracle.cell_areas(c)
    for m in (4, 5):
        assert abs((om * r[m]).sum()) <= 1e-13 * (om * sc[m]).sum()


def _jacobian_sc(u, v, H, k, nx, ny, g=G):
    """Jacobian of the 2-D Euler equations extended by a passive scalar: the
    flux U rho k = (rho k)(n . rho V)/rho differentiated in the conserved
    variables (rho, rho u, rho v, rho E, rho k)."""
    U = nx * u + ny * v
    q2 = u * u + v * v
    ph = 0.5 * (g - 1) * q2
    return np.array([
        [0.0, nx, ny, 0.0, 0.0],
        [nx * ph - u * U, U + u * nx - (g - 1) * u * nx, u * ny - (g - 1) * v * nx, (g - 1) * nx, 0.0],
        [ny * ph - v * U, v * nx - (g - 1) * u * ny, U + v * ny - (g - 1) * v * ny, (g - 1) * ny, 0.0],
        [U * (ph - H), H * nx - (g - 1) * u * U, H * ny - (g - 1) * v * U, g * U, 0.0],
        [-U * k, nx * k, ny * k, 0.0, U],
    ])


@pytest.mark.parametrize("scheme,eps", [(oracle.SCHEME_ROE, None), (oracle.SCHEME_ROE_HARTEN, 0.2)])
def test_classical_roe_scalar_row_equals_eigen_form(scheme, eps):
    WL, WR, nrm = workloads.random_prim_pairs(200, seed=workloads.SEED_BASE + 101)
    rng = np.random.default_rng(5)
    prm = workloads.default_params(scheme=scheme, eps_lambda=eps or 0.1)
    for m in range(200):
        nx, ny = nrm[m]
        kL, kR = rng.uniform(0.1, 2.0, 2)
        wl, wr = np.append(WL[m], kL), np.append(WR[m], kR)
        F = oracle.face_flux_sc(prm, wl, wr, nx, ny)
        _, d = oracle.face_flux(prm, WL[m], WR[m], nx, ny)
        rr = math.sqrt(wr[0] / wl[0])
        khat = (kL + rr * kR) / (1.0 + rr)
        A = _jacobian_sc(d["u"], d["v"], d["H"], khat, nx, ny)
        lam, Rm = np.linalg.eig(A)
        al = np.abs(lam.real)
        if eps is not None:
            h = eps * al.max()
            al = np.where(al < h, 0.5 * (al * al / h + h), al)

        def cons(w):
            rho, u, v, p, k = w
            return np.array([rho, rho * u, rho * v, p / (G - 1) + 0.5 * rho * (u * u + v * v), rho * k])

        def flux(w):
            rho, u, v, p, k = w
            return (nx * u + ny * v) * rho * k

        dQ = cons(wr) - cons(wl)
        diss = (Rm @ np.diag(al) @ np.linalg.solve(Rm, dQ.astype(complex))).real
        ref = 0.5 * (flux(wl) + flux(wr)) - 0.5 * diss[4]
        scale = abs(flux(wl)) + abs(flux(wr)) + abs(F[0]) * max(kL, kR)
        assert abs(F[4] - ref) <= 1e-11 * scale, (m, F[4], ref)


def test_run_with_scalars_keeps_the_flow_and_the_unit_scalar():
    """SSP-RK3 steps: the flow rows are those of the run without scalars, and a
    unit scalar stays equal to the density (bitwise)."""
    base = workloads.smooth_random_case(20, 12, 9, bc=(DIRICHLET, TRANSMISSIVE, SLIPWALL, SLIPWALL), order=2,
                                        eps1=1.0, time_scheme=1)
    c = workloads.add_scalars(base, 2, seed=2)
    c.q0[4] = c.q0[0]  # k_1 = 1
    c.bc_scalar[:, 0] = base.bc_state[:, 0]
    q, st = oracle.run(c, nsteps=5)
    q0, st0 = oracle.run(base, nsteps=5)
    assert np.array_equal(q[:4], q0) and st["t"] == st0["t"]
    assert np.array_equal(q[4], q[0])
    assert np.all(q[5] > 0)
