"""Pins of the 3-D oracle (the paper's equations in their own dimension):
exact reduction to the pinned 2-D oracle on z-invariant states, rotational
invariance of the 3-D flux (the cross products of Eq. 109 and the nine-face
detector included), axis-permutation symmetry of the residual, free stream,
conservation and consistency."""
import math

import numpy as np
import pytest

import oracle
import workloads
from workloads import DIRICHLET, PERIODIC, SLIPWALL, TRANSMISSIVE

G = 1.4


def _rows2(r3):
    return r3[[0, 1, 2, 4]]


@pytest.mark.parametrize("name,c2", [
    ("vortex_eps1", workloads.vortex(32, 0.01)),
    ("smooth_walls_o2", workloads.smooth_random_case(24, 20, 5, bc=(TRANSMISSIVE, DIRICHLET, SLIPWALL, SLIPWALL),
                                                     order=2, eps1=1.0, mach_ref=0.05)),
    ("sod_o1", workloads.sod(nx=60, ny=3)),
])
def test_3d_reduces_to_2d(name, c2):
    """A z-invariant state with w = 0 (periodic in z, dz = 1): every z-slice of
    the 3-D residual is the 2-D residual and the rho w row is zero.  (Runs are
    not compared: the 3-D time-step rule also counts the z faces.)"""
    c3 = workloads.extrude(c2, 3)
    r2, sc = oracle.residual(c2, with_scale=True)
    r3 = oracle.residual3(c3)
    assert np.all(r3[3] == 0.0)
    for l in range(3):
        d = np.abs(_rows2(r3[:, l]) - r2).max(axis=(1, 2)) / sc.max(axis=(1, 2))
        assert np.all(d <= 1e-15), d


def _random_rotation(rng):
    a = rng.normal(size=(3, 3))
    qm, rm = np.linalg.qr(a)
    qm *= np.sign(np.diag(rm))
    if np.linalg.det(qm) < 0:
        qm[:, 0] *= -1
    return qm


@pytest.mark.parametrize("params", [dict(eps1=1.0, mach_ref=0.05), dict(eps1=0.0), dict(scheme=1),
                                    dict(scheme=2, eps_lambda=0.3), dict(eps1=1.0, variant=1 | 2)])
def test_3d_flux_rotation_invariance(params):
    """F(R W, R n) = R F(W, n) for random rotations R (momentum rows rotate,
    the others are unchanged): the 3-D vector algebra, including n1 and the
    cross products of Eq. (109), has no preferred axis."""
    rng = np.random.Generator(np.random.PCG64(workloads.SEED_BASE + 77))
    prm = workloads.default_params(**params)
    for _ in range(200):
        WL = np.array([math.exp(rng.uniform(-1, 1)), *rng.normal(size=3) * 1.5, math.exp(rng.uniform(-1, 1))])
        WR = np.array([math.exp(rng.uniform(-1, 1)), *rng.normal(size=3) * 1.5, math.exp(rng.uniform(-1, 1))])
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        s1 = rng.uniform(0, 1)
        R = _random_rotation(rng)
        F = oracle.face_flux3(prm, WL, WR, n, s1)
        WLr, WRr = WL.copy(), WR.copy()
        WLr[1:4], WRr[1:4] = R @ WL[1:4], R @ WR[1:4]
        Fr = oracle.face_flux3(prm, WLr, WRr, R @ n, s1)
        expect = F.copy()
        expect[1:4] = R @ F[1:4]
        assert np.abs(Fr - expect).max() <= 1e-12 * (1.0 + np.abs(F).max())


def test_3d_flux_consistency_and_symmetry():
    rng = np.random.Generator(np.random.PCG64(workloads.SEED_BASE + 78))
    prm = workloads.default_params(eps1=1.0, mach_ref=0.1)
    for _ in range(100):
        W = np.array([math.exp(rng.uniform(-1, 1)), *rng.normal(size=3), math.exp(rng.uniform(-1, 1))])
        W2 = np.array([math.exp(rng.uniform(-1, 1)), *rng.normal(size=3), math.exp(rng.uniform(-1, 1))])
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        Fp = oracle.physical_flux3(W, n)
        assert np.abs(oracle.face_flux3(prm, W, W, n) - Fp).max() <= 1e-13 * np.abs(Fp).max()
        # swapping the sides and reversing the normal reverses the flux
        F = oracle.face_flux3(prm, W, W2, n)
        Fs = oracle.face_flux3(prm, W2, W, -n)
        assert np.abs(F + Fs).max() <= 1e-12 * np.abs(F).max()


def _permute(q):
    """Relabel the axes x' = y, y' = z, z' = x: cell (i, j, l) becomes
    (i', j', l') = (j, l, i) and (u', v', w') = (v, w, u)."""
    qp = np.ascontiguousarray(np.transpose(q, (0, 3, 1, 2)))
    return qp[[0, 2, 3, 1, 4]]


def test_3d_axis_permutation():
    c = workloads.rough_case3(7, 6, 5, 3, order=2, eps1=1.0, mach_ref=0.05)
    c.dx = c.dy = c.dz = 0.1
    r, sc = oracle.residual3(c, with_scale=True)
    cp = workloads.rough_case3(6, 5, 7, 3, order=2, eps1=1.0, mach_ref=0.05)
    cp.q0 = _permute(c.q0)
    cp.dx = cp.dy = cp.dz = 0.1
    rp = oracle.residual3(cp)
    assert rp.shape == _permute(r).shape
    assert np.abs(rp - _permute(r)).max() <= 1e-13 * sc.max()


@pytest.mark.parametrize("bc", [(PERIODIC,) * 6, (TRANSMISSIVE,) * 6, (DIRICHLET, TRANSMISSIVE) * 3])
def test_3d_free_stream(bc):
    c = workloads.smooth_random_case3(6, 5, 4, 1, bc=bc)
    W = (1.2, 0.3, -0.2, 0.4, 0.8)
    c.q0 = np.ascontiguousarray(np.broadcast_to(workloads.conserved3(G, *W)[:, None, None, None], (5, 4, 5, 6)))
    for s in range(6):
        c.bc_state[s] = workloads.conserved3(G, *W)
    assert np.all(oracle.residual3(c) == 0.0)


def test_3d_conservation_periodic():
    c = workloads.rough_case3(8, 6, 5, 4, order=2, eps1=1.0)
    r, sc = oracle.residual3(c, with_scale=True)
    tot = r.sum(axis=(1, 2, 3))
    mag = sc.sum(axis=(1, 2, 3))
    assert np.all(np.abs(tot) <= 1e-13 * mag)


def test_3d_slip_wall_normal_flux():
    """A slip wall carries no mass or energy: with walls on all six sides the
    totals of the rho and rho E residuals vanish."""
    c = workloads.rough_case3(6, 5, 4, 5, bc=(SLIPWALL,) * 6, order=2, eps1=1.0)
    r, sc = oracle.residual3(c, with_scale=True)
    for k in (0, 4):
        assert abs(r[k].sum()) <= 1e-13 * sc[k].sum()


def test_3d_axis_swap():
    """Swapping x and y (an improper relabelling) also commutes with the
    residual: together with the cyclic permutation this leaves no room for a
    direction-dependent stencil or detector mistake."""
    c = workloads.rough_case3(7, 6, 5, 9, order=2, eps1=1.0, mach_ref=0.05)
    c.dx = c.dy = c.dz = 0.1
    r, sc = oracle.residual3(c, with_scale=True)

    def swap(q):
        qs = np.ascontiguousarray(np.transpose(q, (0, 1, 3, 2)))  # [k][l][i][j]: x' = y, y' = x
        return qs[[0, 2, 1, 3, 4]]

    cs = workloads.rough_case3(6, 7, 5, 9, order=2, eps1=1.0, mach_ref=0.05)
    cs.q0 = swap(c.q0)
    cs.dx = cs.dy = cs.dz = 0.1
    assert np.abs(oracle.residual3(cs) - swap(r)).max() <= 1e-13 * sc.max()
