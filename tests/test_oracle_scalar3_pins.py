"""Pins of the 3-D oracle's transported-scalar rows (Eq. 85 as printed: rows rho,
rho u, rho v, rho w, rho H and rho k).

As in two dimensions, a passive scalar rides on the mass flux: k = 1 gives the
mass row bitwise, k = c gives c times it, and a uniform flow reduces the scheme
to upwind advection of k (a textbook closed form).  A z-invariant state with
scalars gives, in every slice, the pinned 2-D oracle's residual; the classical
Roe row is checked against the eigen-decomposition of the 3-D Roe matrix
extended by the scalar; the scalar rows do not see a rotation of the frame.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from workloads import DIRICHLET, PERIODIC, SLIPWALL, TRANSMISSIVE

G = 1.4
BOTTOM_TOP_WALLS = (PERIODIC, PERIODIC, PERIODIC, PERIODIC, SLIPWALL, DIRICHLET)


def base_cases():
    yield workloads.smooth_random_case3(11, 9, 7, 1, order=2, eps1=1.0, mach_ref=0.05)
    yield workloads.smooth_random_case3(9, 8, 7, 2, bc=(TRANSMISSIVE, DIRICHLET, SLIPWALL, SLIPWALL, PERIODIC,
                                                        PERIODIC), order=2, eps1=1.0)
    yield workloads.smooth_random_case3(8, 7, 9, 3, bc=(DIRICHLET, TRANSMISSIVE) + BOTTOM_TOP_WALLS[2:], order=1)
    yield workloads.rough_case3(8, 7, 6, 4, order=2, eps1=1.0)
    yield workloads.smooth_random_case3(8, 7, 6, 5, order=2, scheme=1)
    yield workloads.smooth_random_case3(8, 7, 6, 6, bc=BOTTOM_TOP_WALLS, order=2, scheme=2, eps_lambda=0.2)
    yield workloads.smooth_random_case3(8, 7, 6, 7, order=2, eps1=1.0, variant=2 | 4 | 64 | 128)


CASES = list(base_cases())


@pytest.mark.parametrize("k", range(len(CASES)))
def test_unit_scalar_row_is_the_mass_row_3d(k):
    c = workloads.add_scalars(CASES[k], 1, mode="const", value=1.0)
    r = oracle.residual3(c)
    assert np.array_equal(r[5], r[0])
    assert np.array_equal(r[:5], oracle.residual3(CASES[k]))  # the flow does not see the scalar


@pytest.mark.parametrize("k", range(len(CASES)))
def test_constant_scalar_scales_the_mass_row_3d(k):
    c = workloads.add_scalars(CASES[k], 1, mode="const", value=0.3)
    r, sc = oracle.residual3(c, with_scale=True)
    assert np.abs(r[5] - 0.3 * r[0]).max() <= 1e-14 * sc[0].max()


@pytest.mark.parametrize("k", range(len(CASES)))
def test_second_scalar_twice_the_first_3d(k):
    c = workloads.add_scalars(CASES[k], 2, seed=k, mode="double")
    r = oracle.residual3(c)
    assert np.array_equal(r[6], 2.0 * r[5])


@pytest.mark.parametrize("name,c2", [
    ("smooth_walls_o2", workloads.smooth_random_case(16, 12, 5, bc=(TRANSMISSIVE, DIRICHLET, SLIPWALL, SLIPWALL),
                                                     order=2, eps1=1.0, mach_ref=0.05)),
    ("periodic_roe", workloads.smooth_random_case(14, 10, 6, order=2, scheme=1)),
    ("sod_o1", workloads.sod(nx=40, ny=3)),
])
def test_3d_scalars_reduce_to_2d(name, c2):
    """A z-invariant state with two rough scalars: every slice of the 3-D
    residual is the 2-D oracle's, scalar rows included."""
    c2s = workloads.add_scalars(c2, 2, seed=11)
    c3 = workloads.extrude(c2s, 3)
    r2, sc = oracle.residual(c2s, with_scale=True)
    r3 = oracle.residual3(c3)
    assert np.all(r3[3] == 0.0)
    for l in range(3):
        d = np.abs(r3[[0, 1, 2, 4, 5, 6], l] - r2).max(axis=(1, 2)) / sc.max(axis=(1, 2))
        assert np.all(d <= 1e-15), d


def _minmod(a, b):
    return np.where(a * b <= 0.0, 0.0, np.sign(a) * np.minimum(np.abs(a), np.abs(b)))


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("mach,sgn,scheme", [(0.3, (1, 1, 1), 0), (0.3, (-1, 1, -1), 0), (1.7, (1, -1, 1), 0),
                                             (0.6, (-1, -1, -1), 1)])
def test_uniform_flow_is_upwind_advection_3d(order, mach, sgn, scheme):
    """Uniform rho, V, p with a rough k: on every face the scalar flux is U rho k
    of the upwind face state, and the flow rows stay at zero."""
    nx, ny, nz = 12, 10, 9
    dx, dy, dz = 0.1, 0.07, 0.13
    rho, p = 1.3, 0.9
    cs = math.sqrt(G * p / rho)
    vel = [sgn[0] * mach * cs * 0.7, sgn[1] * mach * cs * 0.5, sgn[2] * mach * cs * math.sqrt(1 - 0.49 - 0.25)]
    q0 = np.zeros((5, nz, ny, nx))
    q0[:] = workloads.conserved3(G, rho, *vel, p)[:, None, None, None]
    base = workloads.Case3(name="uniform3", q0=q0, params=workloads.default_params(
        order=order, eps1=1.0, mach_ref=0.3, u_ref=mach * cs, scheme=scheme, eps_lambda=0.0),
        bc=(PERIODIC,) * 6, dx=dx, dy=dy, dz=dz)
    c = workloads.add_scalars(base, 1, seed=7, mode="rough")
    r, sc = oracle.residual3(c, with_scale=True)
    k = c.q0[5] / c.q0[0]

    def upwind(kk, vn, axis):
        km1, km2, kp0, kp1 = (np.roll(kk, s, axis=axis) for s in (1, 2, 0, -1))
        if order == 1:
            kl, kr = km1, kp0
        else:
            kl = km1 + 0.5 * _minmod(km1 - km2, kp0 - km1)
            kr = kp0 - 0.5 * _minmod(kp0 - km1, kp1 - kp0)
        return vn * rho * (kl if vn > 0 else kr)

    ref = np.zeros_like(k)
    for axis, (vn, h) in zip((2, 1, 0), ((vel[0], dx), (vel[1], dy), (vel[2], dz))):
        f = upwind(k, vn, axis)
        ref -= (np.roll(f, -1, axis=axis) - f) / h
    assert np.abs(r[5] - ref).max() <= 1e-13 * sc[5].max()
    assert np.abs(r[:5]).max() <= 1e-13 * sc[:5].max()


def test_scalar_conservation_3d():
    c = workloads.add_scalars(workloads.rough_case3(10, 9, 8, 9, order=2, eps1=1.0), 2, seed=3)
    r, sc = oracle.residual3(c, with_scale=True)
    for m in (5, 6):
        assert abs(r[m].sum()) <= 1e-13 * sc[m].sum()


def _random_rotation(rng):
    a = rng.normal(size=(3, 3))
    qm, rm = np.linalg.qr(a)
    qm *= np.sign(np.diag(rm))
    if np.linalg.det(qm) < 0:
        qm[:, 0] *= -1
    return qm


@pytest.mark.parametrize("params", [dict(eps1=1.0, mach_ref=0.05), dict(scheme=1), dict(scheme=2, eps_lambda=0.3)])
def test_scalar_rows_are_rotation_invariant(params):
    rng = np.random.Generator(np.random.PCG64(workloads.SEED_BASE + 79))
    prm = workloads.default_params(**params)
    for _ in range(100):
        WL = np.array([math.exp(rng.uniform(-1, 1)), *rng.normal(size=3) * 1.5, math.exp(rng.uniform(-1, 1)),
                       *rng.uniform(0.1, 2.0, 2)])
        WR = np.array([math.exp(rng.uniform(-1, 1)), *rng.normal(size=3) * 1.5, math.exp(rng.uniform(-1, 1)),
                       *rng.uniform(0.1, 2.0, 2)])
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        s1 = rng.uniform(0, 1)
        R = _random_rotation(rng)
        F = oracle.face_flux3_sc(prm, WL, WR, n, s1)
        assert np.array_equal(F[:5], oracle.face_flux3(prm, WL[:5], WR[:5], n, s1))
        WLr, WRr = WL.copy(), WR.copy()
        WLr[1:4], WRr[1:4] = R @ WL[1:4], R @ WR[1:4]
        Fr = oracle.face_flux3_sc(prm, WLr, WRr, R @ n, s1)
        assert np.abs(Fr[5:] - F[5:]).max() <= 1e-12 * (1.0 + np.abs(F).max())


def _jacobian3_sc(u, v, w, H, k, n, g=G):
    """Jacobian of the 3-D Euler flux through a face of unit normal n, in the
    conserved variables (rho, rho u, rho v, rho w, rho E, rho k), extended by the
    passive-scalar flux U rho k."""
    V = np.array([u, v, w])
    U = float(n @ V)
    q2 = float(V @ V)
    ph = 0.5 * (g - 1) * q2
    A = np.zeros((6, 6))
    A[0, 1:4] = n
    for a in range(3):
        A[1 + a, 0] = n[a] * ph - V[a] * U
        A[1 + a, 1:4] = V[a] * n - (g - 1) * n[a] * V
        A[1 + a, 1 + a] += U
        A[1 + a, 4] = (g - 1) * n[a]
    A[4, 0] = U * (ph - H)
    A[4, 1:4] = H * n - (g - 1) * V * U
    A[4, 4] = g * U
    A[5, 0] = -U * k
    A[5, 1:4] = k * n
    A[5, 5] = U
    return A


@pytest.mark.parametrize("scheme,eps", [(oracle.SCHEME_ROE, None), (oracle.SCHEME_ROE_HARTEN, 0.2)])
def test_classical_roe_3d_scalar_row_equals_eigen_form(scheme, eps):
    """Roe averages (sqrt(rho) weights) of u, v, w, H and k; the upwind
    dissipation |A| dQ of the extended matrix, row rho k, against the oracle."""
    rng = np.random.Generator(np.random.PCG64(workloads.SEED_BASE + 80))
    prm = workloads.default_params(scheme=scheme, eps_lambda=eps or 0.1)

    def cons(w):
        rho, u, v, ww, p, k = w
        return np.array([rho, rho * u, rho * v, rho * ww, p / (G - 1) + 0.5 * rho * (u * u + v * v + ww * ww),
                         rho * k])

    for m in range(150):
        WL = np.array([math.exp(rng.uniform(-1, 1)), *rng.normal(size=3), math.exp(rng.uniform(-1, 1)),
                       rng.uniform(0.1, 2.0)])
        WR = np.array([math.exp(rng.uniform(-1, 1)), *rng.normal(size=3), math.exp(rng.uniform(-1, 1)),
                       rng.uniform(0.1, 2.0)])
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        F = oracle.face_flux3_sc(prm, WL, WR, n, 1.0)
        sl, sr = math.sqrt(WL[0]), math.sqrt(WR[0])

        def avg(a, b):
            return (sl * a + sr * b) / (sl + sr)

        HL = G / (G - 1) * WL[4] / WL[0] + 0.5 * (WL[1:4] @ WL[1:4])
        HR = G / (G - 1) * WR[4] / WR[0] + 0.5 * (WR[1:4] @ WR[1:4])
        A = _jacobian3_sc(*(avg(WL[a], WR[a]) for a in (1, 2, 3)), avg(HL, HR), avg(WL[5], WR[5]), n)
        lam, Rm = np.linalg.eig(A)
        al = np.abs(lam.real)
        if eps is not None:
            h = eps * al.max()
            al = np.where(al < h, 0.5 * (al * al / h + h), al)
        dQ = cons(WR) - cons(WL)
        diss = (Rm @ np.diag(al) @ np.linalg.solve(Rm, dQ.astype(complex))).real
        fl, fr = float(n @ WL[1:4]) * WL[0] * WL[5], float(n @ WR[1:4]) * WR[0] * WR[5]
        ref = 0.5 * (fl + fr) - 0.5 * diss[5]
        scale = abs(fl) + abs(fr) + abs(F[0]) * max(WL[5], WR[5]) + abs(diss[0]) * 2.0
        assert abs(F[5] - ref) <= 1e-11 * scale, (m, F[5], ref)


def test_run3_with_scalars_keeps_the_flow_and_the_unit_scalar():
    base = workloads.smooth_random_case3(10, 8, 7, 9, bc=(DIRICHLET, TRANSMISSIVE, SLIPWALL, SLIPWALL, PERIODIC,
                                                          PERIODIC), order=2, eps1=1.0, time_scheme=1)
    c = workloads.add_scalars(base, 2, seed=2)
    c.q0[5] = c.q0[0]  # k_1 = 1
    c.bc_scalar[:, 0] = base.bc_state[:, 0]
    q, st = oracle.run3(c, nsteps=4)
    q0, st0 = oracle.run3(base, nsteps=4)
    assert np.array_equal(q[:5], q0) and st["t"] == st0["t"]
    assert np.array_equal(q[5], q[0])
    assert np.all(q[6] > 0)
