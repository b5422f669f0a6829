"""Seeded synthetic inputs shaped like the paper's test cases (arXiv 1711.09272, Sec. 7).

This module holds only input generation: grids, initial states, boundary
specifications and request traces.  It contains none of the numerical
method's arithmetic, so it can feed both the CPU oracle and the GPU library,
which otherwise share no code.

A :class:`Case` describes one structured 2-D grid:

* ``q0``: conserved state, float64 array [4 + ns, ny, nx] (rho, rho u, rho v, rho E,
  then ``ns`` transported scalars rho k_m, usually none);
* geometry: uniform ``dx``, ``dy`` or node coordinates ``xn``, ``yn`` [ny+1, nx+1];
* ``bc``: boundary kinds for (west, east, south, north);
* ``bc_state``: conserved Dirichlet state per side [4, 4];
* ``params``: scheme parameters (gamma, CFL, M_ref, U_ref, eps1, eps2, s1 mode,
  reconstruction order, time scheme);
* ``nsteps`` / ``t_end``: run length.
"""
from __future__ import annotations

import dataclasses
import math
from fractions import Fraction
from typing import Dict, List, Optional, Tuple

import numpy as np

SEED_BASE = 171109272

PERIODIC, TRANSMISSIVE, SLIPWALL, DIRICHLET, MOVING = 0, 1, 2, 3, 4
WEST, EAST, SOUTH, NORTH = 0, 1, 2, 3


def default_params(**kw) -> Dict:
    p = dict(gamma=1.4, cfl=0.4, mach_ref=1.0, u_ref=1.0, eps1=0.0, eps2=0.05,
             eps_lambda=0.1, s1_mode=0, order=1, time_scheme=0, scheme=0, variant=0)
    p.update(kw)
    return p


@dataclasses.dataclass
class Case:
    name: str
    q0: np.ndarray
    params: Dict
    bc: Tuple[int, int, int, int]
    dx: float = 1.0
    dy: float = 1.0
    xn: Optional[np.ndarray] = None
    yn: Optional[np.ndarray] = None
    bc_state: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((4, 4)))
    nsteps: int = 1
    t_end: float = 0.0
    bc_scalar: Optional[np.ndarray] = None  # [4 sides, nscalars] Dirichlet rho k_m
    # moving-split sides (kind MOVING): {side: (a, b, hi_kind, conserved state above the split)};
    # below the split point a + b t (cell-centre coordinate along the side) the side's bc_state
    moving: Optional[Dict] = None
    t_bc: float = 0.0  # time at which a residual evaluates moving sides

    @property
    def nscalars(self) -> int:
        return self.q0.shape[0] - 4

    @property
    def ny(self) -> int:
        return self.q0.shape[1]

    @property
    def nx(self) -> int:
        return self.q0.shape[2]

    @property
    def metric(self) -> int:
        return 0 if self.xn is None else 1

    @property
    def cells(self) -> int:
        return self.nx * self.ny


def conserved(gamma: float, rho, u, v, p) -> np.ndarray:
    """Primitive (rho, u, v, p) -> conserved (rho, rho u, rho v, rho E), ideal gas."""
    rho, u, v, p = (np.asarray(a, dtype=np.float64) for a in (rho, u, v, p))
    rhoE = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.stack(np.broadcast_arrays(rho, rho * u, rho * v, rhoE)).astype(np.float64)


def cell_centres(nx: int, ny: int, x0: float, y0: float, dx: float, dy: float):
    x = x0 + (np.arange(nx) + 0.5) * dx
    y = y0 + (np.arange(ny) + 0.5) * dy
    return np.meshgrid(x, y)  # [ny, nx] each


# --------------------------------------------------------------------------
# Shock tubes (Sec. 7.1 and the Sod configuration)
# --------------------------------------------------------------------------

def shock_tube(left, right, x0: float, nx: int = 400, ny: int = 4, t_end: float = 0.2,
               name: str = "shock_tube", **params) -> Case:
    """1-D Riemann problem along x on [0,1] x [0, ny dx]; states are (rho, u, v, p).

    Transmissive in x, periodic in y.  The paper runs its tubes on 200 x 10
    cells with first-order space (Sec. 7.1)."""
    dx = 1.0 / nx
    X, _ = cell_centres(nx, ny, 0.0, 0.0, dx, dx)
    gamma = params.get("gamma", 1.4)
    st = [np.where(X < x0, left[k], right[k]) for k in range(4)]
    q0 = conserved(gamma, *st)
    prm = default_params(order=1, time_scheme=0, eps1=0.0, s1_mode=0, mach_ref=1.0, u_ref=1.0)
    prm.update(params)
    return Case(name=name, q0=q0, params=prm, bc=(TRANSMISSIVE, TRANSMISSIVE, PERIODIC, PERIODIC),
                dx=dx, dy=dx, nsteps=100000, t_end=t_end)


def sod(nx: int = 400, ny: int = 4, **params) -> Case:
    """Sod tube: (1, 0, 0, 1) | (0.125, 0, 0, 0.1) at x = 0.5, first order, forward
    Euler, CFL 0.4, to t = 0.2 (first test configuration)."""
    return shock_tube((1.0, 0.0, 0.0, 1.0), (0.125, 0.0, 0.0, 0.1), 0.5, nx, ny, 0.2,
                      name=f"sod_{nx}x{ny}", **params)


# The shock tubes of Sec. 7.1 in the paper's own setting: 200 x 10 cells,
# first order in space, the four-stage Runge-Kutta scheme, eps1 = 0, and
# s1 = 1 of Eq. (110) (reading: with M_ref = 1 nothing is preconditioned,
# theta = 1, so these problems hold no low-Mach, large-pressure-gradient flow
# for the detector of Eqs. 95-97 to guard against).  The paper prints no CFL
# number; 0.4 is ours.
SEC71_SETTING = dict(order=1, time_scheme=2, eps1=0.0, s1_mode=1)


def expansion_shock_tube(nx: int = 200, ny: int = 10, **params) -> Case:
    """Sec. 7.1.1: (3, 0.9, 0, 3) | (1, 0.9, 0, 1) at 0.3, t = 0.2."""
    return shock_tube((3.0, 0.9, 0.0, 3.0), (1.0, 0.9, 0.0, 1.0), 0.3, nx, ny, 0.2,
                      name="expansion_shock", **dict(SEC71_SETTING, **params))


def near_vacuum_tube(nx: int = 200, ny: int = 10, **params) -> Case:
    """Sec. 7.1.2: (1, -2, 0, 0.4) | (1, 2, 0, 0.4) at 0.5, t = 0.15."""
    return shock_tube((1.0, -2.0, 0.0, 0.4), (1.0, 2.0, 0.0, 0.4), 0.5, nx, ny, 0.15,
                      name="near_vacuum", **dict(SEC71_SETTING, **params))


def strong_shock_tube(nx: int = 200, ny: int = 10, **params) -> Case:
    """Sec. 7.1.3: (1, 0, 0, 1000) | (1, 0, 0, 0.01) at 0.5, t = 0.012."""
    return shock_tube((1.0, 0.0, 0.0, 1000.0), (1.0, 0.0, 0.0, 0.01), 0.5, nx, ny, 0.012,
                      name="strong_shock", **dict(SEC71_SETTING, **params))


# --------------------------------------------------------------------------
# Moving normal shock (Rankine-Hugoniot), exact rationals
# --------------------------------------------------------------------------

def moving_shock_state(mach, rho1=Fraction(7, 5), p1=Fraction(1), gamma=Fraction(7, 5)):
    """Post-shock (rho2, u2, p2) of a normal shock of Mach ``mach`` moving into gas at rest.

    Textbook normal-shock relations, evaluated in exact rational arithmetic when
    the inputs are rationals (the Sec. 7.2 state is printed as rationals)."""
    M2 = Fraction(mach) ** 2
    g = Fraction(gamma)
    p2 = p1 * (1 + 2 * g / (g + 1) * (M2 - 1))
    rho2 = rho1 * (g + 1) * M2 / ((g - 1) * M2 + 2)
    c1_sq = g * p1 / rho1
    # u2 = Ms c1 (1 - rho1/rho2); c1 is rational here when c1^2 is a square.
    num, den = c1_sq.numerator, c1_sq.denominator
    rn, rd = math.isqrt(num), math.isqrt(den)
    if rn * rn == num and rd * rd == den:
        c1 = Fraction(rn, rd)
    else:
        c1 = Fraction(math.sqrt(float(c1_sq)))
    u2 = Fraction(mach) * c1 * (1 - rho1 / rho2)
    return rho2, u2, p2


# --------------------------------------------------------------------------
# Low-Mach isentropic vortex (second test configuration)
# --------------------------------------------------------------------------

def vortex(n: int = 256, mach: float = 0.01, stationary: bool = False, seed: Optional[int] = None,
           checker_amp: float = 1e-6, nsteps: int = 1000, **params) -> Case:
    """Isentropic vortex on [0,10]^2, periodic, rho_inf = p_inf = 1 (c_inf = sqrt(gamma)).

    Free stream M c_inf (1,1)/sqrt(2), or at rest when ``stationary``.  Vortex
    strength beta = 5 M c_inf so the pressure dip scales with M^2.  The
    pressure is then multiplied by 1 + checker_amp (-1)^(i+j) u_ij with u_ij
    uniform in [0.5, 1.5) from the seed: a seeded checkerboard."""
    gamma = params.get("gamma", 1.4)
    seed = SEED_BASE + 1 if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    L = 10.0
    dx = L / n
    X, Y = cell_centres(n, n, 0.0, 0.0, dx, dx)
    cinf = math.sqrt(gamma)
    beta = 5.0 * mach * cinf
    vinf = 0.0 if stationary else mach * cinf / math.sqrt(2.0)
    xr, yr = X - 5.0, Y - 5.0
    r2 = xr * xr + yr * yr
    amp = beta / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
    u = vinf - amp * yr
    v = vinf + amp * xr
    T = 1.0 - (gamma - 1.0) * beta * beta / (8.0 * gamma * math.pi ** 2) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    I, J = np.meshgrid(np.arange(n), np.arange(n))
    chk = np.where((I + J) % 2 == 0, 1.0, -1.0)
    p = p * (1.0 + checker_amp * chk * rng.uniform(0.5, 1.5, size=(n, n)))
    q0 = conserved(gamma, rho, u, v, p)
    u_ref = math.sqrt(2.0) * vinf if not stationary else mach * cinf
    prm = default_params(order=2, time_scheme=1, cfl=0.4, mach_ref=mach, u_ref=u_ref,
                         eps1=1.0, eps2=0.05, s1_mode=0)
    prm.update(params)
    return Case(name=f"vortex_{n}_M{mach:g}{'_rest' if stationary else ''}", q0=q0, params=prm,
                bc=(PERIODIC,) * 4, dx=dx, dy=dx, nsteps=nsteps, t_end=0.0)


# --------------------------------------------------------------------------
# Hypersonic odd-even decoupling (third test configuration; Sec. 7.2)
# --------------------------------------------------------------------------

def odd_even(nx: int = 800, ny: int = 80, mach: float = 20.0, eps_y: float = 1e-6,
             seeded: bool = True, seed: Optional[int] = None, shock_x: float = 20.0,
             t_end: float = 30.0, **params) -> Case:
    """Planar Mach-``mach`` shock moving into (rho, p) = (1.4, 1) in an nx x ny
    channel of unit cells.  The centreline node row is displaced by
    +-eps_y cell heights: alternating in i as in Eq. (113), or with a seeded
    sign per node column.  Left: Dirichlet post-shock inflow; right:
    transmissive; top and bottom: slip walls."""
    gamma = params.get("gamma", 1.4)
    seed = SEED_BASE + 2 if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    xs = np.arange(nx + 1, dtype=np.float64)
    ys = np.arange(ny + 1, dtype=np.float64)
    xn, yn = np.meshgrid(xs, ys)
    jmid = ny // 2
    if seeded:
        s = rng.choice(np.array([-1.0, 1.0]), size=nx + 1)
    else:
        s = np.where(np.arange(nx + 1) % 2 == 0, 1.0, -1.0)
    yn = yn.copy()
    yn[jmid, :] = jmid + eps_y * s
    rho2, u2, p2 = (float(v) for v in moving_shock_state(Fraction(mach).limit_denominator(10 ** 6)))
    X, _ = cell_centres(nx, ny, 0.0, 0.0, 1.0, 1.0)
    post = (rho2, u2, 0.0, p2)
    pre = (1.4, 0.0, 0.0, 1.0)
    st = [np.where(X < shock_x, post[k], pre[k]) for k in range(4)]
    q0 = conserved(gamma, *st)
    bc_state = np.zeros((4, 4))
    bc_state[WEST] = conserved(gamma, *post)
    prm = default_params(order=2, time_scheme=1, cfl=0.4, mach_ref=1.0, u_ref=u2,
                         eps1=1.0, eps2=0.05, s1_mode=0)
    prm.update(params)
    return Case(name=f"odd_even_{nx}x{ny}_M{mach:g}", q0=q0, params=prm,
                bc=(DIRICHLET, TRANSMISSIVE, SLIPWALL, SLIPWALL), xn=xn, yn=yn,
                bc_state=bc_state, nsteps=100000, t_end=t_end)


# --------------------------------------------------------------------------
# Body-fitted O-grids around a circular cylinder (Secs. 7.5 and 7.6)
# --------------------------------------------------------------------------

def cylinder_ogrid(n_circ: int, n_rad: int, r_in: float = 1.0, r_out: float = 4.0, ratio: float = 1.0,
                   half: bool = False):
    """Nodes of an O-grid around a cylinder of radius r_in centred at the origin:
    i runs clockwise around the circumference (n_circ cells; node column n_circ
    coincides with column 0, so the i direction is periodic), j outward
    (n_rad cells) with radial spacing growing geometrically by ``ratio`` per
    cell.  Clockwise i and outward j make the cells positively oriented for the
    face-vector convention of the solver.  half=True: only the upstream half
    (x <= 0), from the bottom (theta = -90 deg) clockwise to the top.  Returns
    xn, yn of shape (n_rad + 1, n_circ + 1)."""
    if ratio == 1.0:
        w = np.arange(n_rad + 1, dtype=np.float64) / n_rad
    else:
        w = (ratio ** np.arange(n_rad + 1, dtype=np.float64) - 1.0) / (ratio ** n_rad - 1.0)
    r = r_in + (r_out - r_in) * w
    if half:
        th = -0.5 * math.pi - math.pi * np.arange(n_circ + 1, dtype=np.float64) / n_circ
    else:
        th = -2.0 * math.pi * np.arange(n_circ + 1, dtype=np.float64) / n_circ
    R, TH = np.meshgrid(r, th, indexing="ij")
    xn, yn = R * np.cos(TH), R * np.sin(TH)
    if half:
        xn[:, 0] = xn[:, -1] = 0.0  # the cut along the y axis, exactly
    else:
        xn[:, -1], yn[:, -1] = xn[:, 0], yn[:, 0]  # close the ring exactly
    return xn, yn


def _node_centres(xn, yn):
    return 0.25 * (xn[:-1, :-1] + xn[:-1, 1:] + xn[1:, :-1] + xn[1:, 1:]), \
        0.25 * (yn[:-1, :-1] + yn[:-1, 1:] + yn[1:, :-1] + yn[1:, 1:])


def cylinder_carbuncle(n_circ: int = 160, n_rad: int = 20, mach: float = 20.0, r_out: float = 2.0,
                       jitter: float = 0.0, seed: Optional[int] = None, **params) -> Case:
    """Sec. 7.5: Mach-20 flow (rho = 1.4, p = 1, so c = 1) past a unit cylinder on
    160 x 20 cells (circumference x radius) of the upstream half O-grid (the
    bow-shock region; the near-vacuum wake is outside the domain, as in the
    usual form of this test); slip wall on the cylinder, free-stream Dirichlet
    state on the outer arc, transmissive (supersonic outflow) cuts at the top
    and bottom; impulsive start from the free stream.  First order, forward
    Euler (the paper's shock tests use a first-order space discretisation)."""
    gamma = params.get("gamma", 1.4)
    xn, yn = cylinder_ogrid(n_circ, n_rad, 1.0, r_out, half=True)
    if jitter:
        # seeded displacement of the interior nodes along the radius, a fraction
        # ``jitter`` of the radial spacing (the seed of a shock instability)
        rng = np.random.Generator(np.random.PCG64(SEED_BASE + 5 if seed is None else seed))
        f = 1.0 + jitter * (r_out - 1.0) / n_rad * rng.uniform(-1.0, 1.0, xn.shape) / np.hypot(xn, yn)
        f[0, :] = f[-1, :] = 1.0
        xn, yn = xn * f, yn * f
    ny, nx = n_rad, n_circ
    fs = (1.4, mach, 0.0, 1.0)
    q0 = conserved(gamma, *[np.full((ny, nx), v) for v in fs])
    bc_state = np.zeros((4, 4))
    bc_state[NORTH] = conserved(gamma, *fs)
    prm = default_params(order=1, time_scheme=0, cfl=0.4, mach_ref=1.0, u_ref=mach, eps1=0.0, eps2=0.05,
                         s1_mode=0)
    prm.update(params)
    return Case(name=f"carbuncle_{nx}x{ny}", q0=q0, params=prm, bc=(TRANSMISSIVE, TRANSMISSIVE, SLIPWALL, DIRICHLET),
                xn=xn, yn=yn, bc_state=bc_state, nsteps=1000, t_end=0.0)


def cylinder_potential_state(xn, yn, mach: float, gamma: float = 1.4):
    """Incompressible potential flow past the unit cylinder, free stream along +x
    (rho = 1, p = 1/gamma, so c = 1 and U = mach), pressure from Bernoulli's
    law, evaluated at the cell centres of the O-grid."""
    X, Y = _node_centres(xn, yn)
    r2 = X * X + Y * Y
    th = np.arctan2(Y, X)
    ur = mach * (1.0 - 1.0 / r2) * np.cos(th)
    ut = -mach * (1.0 + 1.0 / r2) * np.sin(th)
    u = ur * np.cos(th) - ut * np.sin(th)
    v = ur * np.sin(th) + ut * np.cos(th)
    rho = np.ones_like(u)
    p = 1.0 / gamma + 0.5 * (mach * mach - (u * u + v * v))
    return conserved(gamma, rho, u, v, p)


def cylinder_low_mach(n_circ: int = 100, n_rad: int = 72, mach: float = 0.01, r_out: float = 20.0,
                      ratio: float = 1.06, **params) -> Case:
    """Sec. 7.6: low-Mach inviscid flow past a unit cylinder on a 100 x 72 O-grid
    (circumference x radius, radial spacing stretched), slip wall on the
    cylinder, free-stream Dirichlet state on the outer circle, started from
    the incompressible potential flow.  MUSCL + SSP-RK3, M_ref = the inlet
    Mach number."""
    gamma = params.get("gamma", 1.4)
    xn, yn = cylinder_ogrid(n_circ, n_rad, 1.0, r_out, ratio)
    q0 = cylinder_potential_state(xn, yn, mach, gamma)
    bc_state = np.zeros((4, 4))
    bc_state[NORTH] = conserved(gamma, 1.0, mach, 0.0, 1.0 / gamma)
    prm = default_params(order=2, time_scheme=1, cfl=0.4, mach_ref=mach, u_ref=mach, eps1=1.0, eps2=0.05,
                         s1_mode=0)
    prm.update(params)
    return Case(name=f"cylinder_{n_circ}x{n_rad}_M{mach:g}", q0=q0, params=prm,
                bc=(PERIODIC, PERIODIC, SLIPWALL, DIRICHLET), xn=xn, yn=yn, bc_state=bc_state, nsteps=100,
                t_end=0.0)


# --------------------------------------------------------------------------
# Batched / serving family (fourth and fifth test configurations)
# --------------------------------------------------------------------------

def bump_spec(rng: np.random.Generator, mach_lo: float = 0.001, mach_hi: float = 20.0) -> Dict:
    """Seeded parameters of one bump-family state: Mach ~ U(lo, hi), direction ~
    U(0, 2 pi), 1-5 Gaussian bumps (centre, sigma ~ U(0.03, 0.1), amplitude ~
    U(0.01, 0.2) with a random sign, target 0 = rho, 1 = p, 2 = both)."""
    mach = rng.uniform(mach_lo, mach_hi)
    ang = rng.uniform(0.0, 2.0 * math.pi)
    bumps = []
    for _ in range(int(rng.integers(1, 6))):
        cx, cy = rng.uniform(0.0, 1.0, size=2)
        sig = rng.uniform(0.03, 0.1)
        a = rng.uniform(0.01, 0.2) * rng.choice(np.array([-1.0, 1.0]))
        bumps.append((float(cx), float(cy), float(sig), float(a), int(rng.integers(0, 3))))
    return {"mach": float(mach), "angle": float(ang), "bumps": bumps}


def bump_fields(n: int, spec: Dict, xp=np, device=None, gamma: float = 1.4):
    """Primitive fields of a bump-family state on [0,1]^2 (rho = 1, p = 1/gamma,
    so c = 1), with xp = numpy or torch (device arrays)."""
    kw = {} if xp is np else {"device": device, "dtype": xp.float64}
    dx = 1.0 / n
    c = (xp.arange(n, **kw) + 0.5) * dx
    Y, X = xp.meshgrid(c, c, indexing="ij")
    rho = xp.ones((n, n), **kw)
    p = xp.full((n, n), 1.0 / gamma, **kw)
    for cx, cy, sig, a, target in spec["bumps"]:
        ddx = xp.abs(X - cx)
        ddx = xp.minimum(ddx, 1.0 - ddx)
        ddy = xp.abs(Y - cy)
        ddy = xp.minimum(ddy, 1.0 - ddy)
        bump = 1.0 + a * xp.exp(-(ddx * ddx + ddy * ddy) / (2.0 * sig * sig))
        if target in (0, 2):
            rho = rho * bump
        if target in (1, 2):
            p = p * bump
    u = xp.full((n, n), spec["mach"] * math.cos(spec["angle"]), **kw)
    v = xp.full((n, n), spec["mach"] * math.sin(spec["angle"]), **kw)
    return rho, u, v, p


def bump_state(n: int, rng: np.random.Generator, gamma: float = 1.4, mach_lo: float = 0.001,
               mach_hi: float = 20.0):
    """Uniform flow on [0,1]^2 (rho = 1, p = 1/gamma so c = 1) times 1-5
    multiplicative Gaussian bumps (minimum-image distance); see bump_spec."""
    spec = bump_spec(rng, mach_lo, mach_hi)
    return conserved(gamma, *bump_fields(n, spec, gamma=gamma)), spec["mach"]


def bump_state_device(n: int, spec: Dict, pitch: int, device="cuda", gamma: float = 1.4):
    """The same state built directly on the GPU with torch, in a padded
    [4, n, pitch] layout (for serving traces with large grids)."""
    import torch
    rho, u, v, p = bump_fields(n, spec, xp=torch, device=device, gamma=gamma)
    out = torch.zeros((4, n, pitch), dtype=torch.float64, device=device)
    out[0, :, :n] = rho
    out[1, :, :n] = rho * u
    out[2, :, :n] = rho * v
    out[3, :, :n] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return out


def bump_params(spec_mach: float, **params) -> Dict:
    prm = default_params(order=2, time_scheme=1, cfl=0.4, mach_ref=min(spec_mach, 1.0), u_ref=spec_mach,
                         eps1=1.0, eps2=0.05, s1_mode=0)
    prm.update(params)
    return prm


def bump_case(n: int, rng: np.random.Generator, nsteps: int, name: str = "bump", **params) -> Case:
    q0, mach = bump_state(n, rng)
    return Case(name=name, q0=q0, params=bump_params(mach, **params), bc=(PERIODIC,) * 4, dx=1.0 / n,
                dy=1.0 / n, nsteps=nsteps, t_end=0.0)


def batch_family(n_grids: int = 256, seed: Optional[int] = None, nsteps: int = 200,
                 n_lo: int = 32, n_hi: int = 512, **params) -> List[Case]:
    """Square grids with side round(exp(U(ln n_lo, ln n_hi)))."""
    seed = SEED_BASE + 3 if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for g in range(n_grids):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        out.append(bump_case(n, rng, nsteps, name=f"batch{g}_{n}", **params))
    return out


def serving_trace(rate: float, duration: float, seed: Optional[int] = None, n_lo: int = 64,
                  n_hi: int = 2048, s_lo: int = 50, s_hi: int = 2000):
    """Poisson arrivals at ``rate`` per second for ``duration`` seconds; each request
    has a square grid side log-uniform in [n_lo, n_hi], a step count log-uniform
    in [s_lo, s_hi] and a bump-family state (bump_spec).  Returns a list of
    dicts (arrival_s, n, steps, spec)."""
    seed = SEED_BASE + 4 if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        s = int(round(math.exp(rng.uniform(math.log(s_lo), math.log(s_hi)))))
        out.append({"arrival_s": t, "n": n, "steps": s, "spec": bump_spec(rng)})
    return out


# --------------------------------------------------------------------------
# Random face states and smooth fields for unit and parity tests
# --------------------------------------------------------------------------

def random_prim_pairs(n: int, seed: int, mach_lo: float = 1e-3, mach_hi: float = 5.0,
                      jump: float = 0.5) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """n pairs of primitive states (rho, u, v, p) and unit normals [n, 2]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rho = np.exp(rng.uniform(-1.0, 1.0, n))
    p = np.exp(rng.uniform(-1.0, 1.0, n))
    c = np.sqrt(1.4 * p / rho)
    mach = np.exp(rng.uniform(math.log(mach_lo), math.log(mach_hi), n))
    ang = rng.uniform(0, 2 * math.pi, n)
    u, v = mach * c * np.cos(ang), mach * c * np.sin(ang)
    WL = np.stack([rho, u, v, p], axis=1)
    f = np.exp(rng.uniform(-jump, jump, (n, 4)))
    WR = WL.copy()
    WR[:, 0] *= f[:, 0]
    WR[:, 3] *= f[:, 3]
    WR[:, 1] += (f[:, 1] - 1.0) * c * mach
    WR[:, 2] += (f[:, 2] - 1.0) * c * mach
    th = rng.uniform(0, 2 * math.pi, n)
    nrm = np.stack([np.cos(th), np.sin(th)], axis=1)
    return WL, WR, nrm


def smooth_random_case(nx: int, ny: int, seed: int, bc=(PERIODIC,) * 4, mach: float = 0.5,
                       amp: float = 0.2, nodes: bool = False, **params) -> Case:
    """A smooth random periodic-like field (sums of a few sines) with mild
    density/pressure variation; optionally on a randomly perturbed node grid."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gamma = params.get("gamma", 1.4)
    dx, dy = 1.0 / nx, 1.0 / ny
    X, Y = cell_centres(nx, ny, 0.0, 0.0, dx, dy)

    def field():
        out = np.zeros_like(X)
        for _ in range(3):
            kx, ky = rng.integers(1, 4, size=2)
            ph = rng.uniform(0, 2 * math.pi)
            out += rng.uniform(-1, 1) * np.sin(2 * math.pi * (kx * X + ky * Y) + ph)
        return out / 3.0

    rho = 1.0 + amp * field()
    p = 1.0 / gamma * (1.0 + amp * field())
    u = mach * (1.0 + field())
    v = mach * field()
    q0 = conserved(gamma, rho, u, v, p)
    xn = yn = None
    if nodes:
        xs = np.arange(nx + 1) * dx
        ys = np.arange(ny + 1) * dy
        xn, yn = np.meshgrid(xs, ys)
        # node perturbation that repeats with the domain period, so opposite
        # boundary faces coincide under the periodic index wrap
        px = 0.15 * dx * rng.uniform(-1, 1, xn.shape)
        py = 0.15 * dy * rng.uniform(-1, 1, yn.shape)
        for a in (px, py):
            a[:, -1] = a[:, 0]
            a[-1, :] = a[0, :]
        xn = xn + px
        yn = yn + py
    prm = default_params(order=2, time_scheme=1, mach_ref=0.1, u_ref=mach, eps1=1.0)
    prm.update(params)
    bc_state = np.zeros((4, 4))
    for s in range(4):
        bc_state[s] = conserved(gamma, 1.0, mach, 0.0, 1.0 / gamma)
    return Case(name=f"smooth_{nx}x{ny}", q0=q0, params=prm, bc=tuple(bc), dx=dx, dy=dy,
                xn=xn, yn=yn, bc_state=bc_state, nsteps=10, t_end=0.0)


def dmr_states(gamma: float = 1.4):
    """Pre- and post-shock primitive states (rho, u, v, p) of the Mach-10 shock of
    the double-Mach reflection: pre (1.4, 0, 0, 1); post from the normal-shock
    relations at gamma = 1.4 (exact: rho = 8, p = 233/2, speed 33/4 along the
    shock normal (cos 30, -sin 30))."""
    w2 = 8.25
    return (1.4, 0.0, 0.0, 1.0), (8.0, w2 * math.cos(math.pi / 6), -w2 * 0.5, 116.5)


def dmr(nx: int = 800, ny: int = 200, t_end: float = 0.2, **params) -> Case:
    """Double-Mach reflection (Sec. 7.4): [0, 4] x [0, 1], a Mach-10 shock at 60
    degrees to the wall through (1/6, 0) moving into (1.4, 0, 0, 1); post-shock
    inflow on the left, transmissive right; the bottom is post-shock for
    x < 1/6 and a slip wall beyond; the top follows the exact shock,
    x_s(t) = 1/6 + (1 + 20 t) / sqrt(3) (post-shock left of it).  200 x 800 cells
    by default (the paper's grid, read as 800 in x and 200 in y, dx = dy = 1/200)."""
    gamma = params.get("gamma", 1.4)
    pre, post = dmr_states(gamma)
    dx, dy = 4.0 / nx, 1.0 / ny
    X, Y = cell_centres(nx, ny, 0.0, 0.0, dx, dy)
    behind = X < 1.0 / 6.0 + Y / math.sqrt(3.0)
    q0 = np.where(behind[None], conserved(gamma, *post)[:, None, None], conserved(gamma, *pre)[:, None, None])
    bc_state = np.zeros((4, 4))
    qpost, qpre = conserved(gamma, *post), conserved(gamma, *pre)
    for sd in range(4):
        bc_state[sd] = qpost
    prm = default_params(order=2, time_scheme=1, cfl=0.4, mach_ref=1.0, u_ref=8.25, eps1=1.0, eps2=0.05)
    prm.update(params)
    moving = {SOUTH: (1.0 / 6.0, 0.0, SLIPWALL, qpost), NORTH: (1.0 / 6.0 + 1.0 / math.sqrt(3.0),
                                                                20.0 / math.sqrt(3.0), DIRICHLET, qpre)}
    return Case(name=f"dmr_{nx}x{ny}", q0=np.ascontiguousarray(q0), params=prm,
                bc=(DIRICHLET, TRANSMISSIVE, MOVING, MOVING), dx=dx, dy=dy, bc_state=bc_state, nsteps=10 ** 6,
                t_end=t_end, moving=moving)


def corner_states():
    """Pre- and post-shock primitive states (rho, u, v, p) of the supersonic corner
    (Sec. 7.3, as printed): the shock moves at rho_L u_L / (rho_L - rho_R) = 5.09
    into gas at rest."""
    return (1.4, 0.0, 0.0, 1.0), (7.04108, 4.07794, 0.0, 30.05942)


def corner(n: int = 400, t_end: float = 0.155, **params) -> Case:
    """Supersonic corner (Sec. 7.3) on the paper's n x n grid of [0, 1]^2 with the
    90-degree corner at (0.05, 0.5) and the shock at x = 0.05.  The inflow channel
    x < 0.05, y > 0.5 holds the post-shock state, which is supersonic (u = 4.08 >
    c = 2.44), so nothing travels upstream into it and it stays uniform; the case
    is therefore the block x > 0.05 (0.95 n x n cells) whose west side is the
    step's slip wall below y = 0.5 and post-shock inflow above it.  East, south
    and north sides are transmissive.  Gas at rest (1.4, 0, 0, 1) fills the block
    at t = 0.  The paper's setting of its Sec. 7 tests: first order in space, the
    four-stage Runge-Kutta scheme, eps1 = 0 unless stated (Fig. 8f: eps1 = 1,
    eps2 = 0.05)."""
    assert n % 20 == 0, "the corner must fall on a cell face"
    gamma = params.get("gamma", 1.4)
    pre, post = corner_states()
    nx, ny = (19 * n) // 20, n
    dx = dy = 1.0 / n
    qpre, qpost = conserved(gamma, *pre), conserved(gamma, *post)
    q0 = np.ascontiguousarray(np.broadcast_to(qpre[:, None, None], (4, ny, nx)))
    bc_state = np.zeros((4, 4))
    bc_state[WEST] = qpost
    prm = default_params(order=1, time_scheme=2, cfl=0.4, mach_ref=1.0, u_ref=post[1], eps1=0.0, eps2=0.05)
    prm.update(params)
    moving = {WEST: (0.5, 0.0, DIRICHLET, qpost, SLIPWALL)}
    return Case(name=f"corner_{nx}x{ny}", q0=q0, params=prm, bc=(MOVING, TRANSMISSIVE, TRANSMISSIVE, TRANSMISSIVE),
                dx=dx, dy=dy, bc_state=bc_state, nsteps=10 ** 6, t_end=t_end, moving=moving)


def add_scalars(case: "Case", ns: int, seed: int = 0, mode: str = "rough", value: float = 1.0,
                k_bc: Optional[np.ndarray] = None) -> "Case":
    """The case with ``ns`` transported scalars appended (rows rho k_m):
    mode "rough": k_m ~ U(0.1, 2) cell by cell; "smooth": a seeded Fourier field in
    (0.2, 1.8); "const": k_m = value everywhere (also on Dirichlet sides); "double":
    two scalars with k_2 = 2 k_1, k_1 rough.  Dirichlet sides carry k_bc[side, m]
    (default: value) times their density."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 600 + seed))
    rho = case.q0[0]
    nsides = len(case.bc)  # 4 in 2-D, 6 in 3-D (a Case3 works as well)
    ks = []
    for m in range(ns):
        if mode == "const":
            k = np.full_like(rho, value)
        elif mode == "smooth":
            idx = np.meshgrid(*(np.arange(n) for n in rho.shape), indexing="ij")
            ph = rng.uniform(0, 2 * math.pi, rho.ndim)
            nd = rho.ndim  # axis nd-1 is x; phases go x, y, z
            k = 0.8 * np.sin(2 * math.pi * idx[nd - 1] / rho.shape[nd - 1] + ph[0])
            for d in range(nd - 2, -1, -1):
                k = k * np.cos(2 * math.pi * idx[d] / rho.shape[d] + ph[nd - 1 - d])
            k = 1.0 + k
        elif mode == "double":
            k = rng.uniform(0.1, 2.0, rho.shape) if m == 0 else 2.0 * ks[0]
        else:
            k = rng.uniform(0.1, 2.0, rho.shape)
        ks.append(k)
    c = dataclasses.replace(case)
    c.q0 = np.concatenate([case.q0, np.stack([rho * k for k in ks])]) if ns else case.q0.copy()
    bcs = np.zeros((nsides, max(ns, 1)))
    for sd in range(nsides):
        for m in range(ns):
            kb = value if k_bc is None else k_bc[sd][m]
            if mode == "double" and m == 1 and k_bc is None:
                kb = 2.0 * value
            bcs[sd, m] = case.bc_state[sd][0] * kb
    c.bc_scalar = bcs[:, :ns] if ns else None
    c.name = f"{case.name}_sc{ns}{mode}"
    return c


# --------------------------------------------------------------------------
# 3-D uniform Cartesian grids
# --------------------------------------------------------------------------
BOTTOM, TOP = 4, 5


@dataclasses.dataclass
class Case3:
    name: str
    q0: np.ndarray               # [5][nz][ny][nx], rows rho, rho u, rho v, rho w, rho E
    params: Dict
    bc: Tuple[int, int, int, int, int, int]
    dx: float = 1.0
    dy: float = 1.0
    dz: float = 1.0
    bc_state: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((6, 5)))
    nsteps: int = 1
    t_end: float = 0.0
    bc_scalar: Optional[np.ndarray] = None  # [6 sides, nscalars] Dirichlet rho k_m

    @property
    def nz(self) -> int:
        return self.q0.shape[1]

    @property
    def ny(self) -> int:
        return self.q0.shape[2]

    @property
    def nx(self) -> int:
        return self.q0.shape[3]

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz


def conserved3(gamma: float, rho, u, v, w, p) -> np.ndarray:
    rho, u, v, w, p = np.broadcast_arrays(*(np.asarray(a, dtype=np.float64) for a in (rho, u, v, w, p)))
    return np.stack([rho, rho * u, rho * v, rho * w, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)])


def smooth_random_case3(nx: int, ny: int, nz: int, seed: int, bc=(PERIODIC,) * 6, mach: float = 0.5,
                        amp: float = 0.2, **params) -> Case3:
    """Smooth periodic-consistent random field on [0,1]^3: a few Fourier modes
    per variable, Mach about ``mach`` in a random direction."""
    gamma = params.get("gamma", 1.4)
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 300 + seed))
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    z = (np.arange(nz) + 0.5) / nz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")

    def field():
        out = np.zeros_like(X)
        for _ in range(3):
            kx, ky, kz = rng.integers(1, 3, size=3)
            ph = rng.uniform(0, 2 * math.pi, size=3)
            out += (rng.uniform(-1, 1) * np.sin(2 * math.pi * kx * X + ph[0]) * np.cos(2 * math.pi * ky * Y + ph[1])
                    * np.cos(2 * math.pi * kz * Z + ph[2]))
        return out / 3.0

    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    rho = 1.0 + amp * field()
    p = 1.0 / gamma * (1.0 + amp * field())
    u, v, w = (mach * d[k] + amp * mach * field() for k in range(3))
    q0 = conserved3(gamma, rho, u, v, w, p)
    prm = default_params(order=2, eps1=1.0, mach_ref=max(mach, 1e-3), u_ref=mach)
    prm.update(params)
    bc_state = np.zeros((6, 5))
    for s in range(6):
        bc_state[s] = conserved3(gamma, 1.0, mach * d[0], mach * d[1], mach * d[2], 1.0 / gamma)
    return Case3(name=f"smooth3_{nx}x{ny}x{nz}", q0=q0, params=prm, bc=tuple(bc), dx=1.0 / nx, dy=1.0 / ny,
                 dz=1.0 / nz, bc_state=bc_state, nsteps=1)


def rough_case3(nx: int, ny: int, nz: int, seed: int, bc=(PERIODIC,) * 6, **params) -> Case3:
    """Cell-by-cell random states: density and pressure over two decades, Mach up
    to 3 in random 3-D directions (limiter, detector and supersonic branches)."""
    c = smooth_random_case3(nx, ny, nz, seed, bc=bc, **params)
    gamma = c.params.get("gamma", 1.4)
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 400 + seed))
    shp = (nz, ny, nx)
    rho = np.exp(rng.uniform(-2.3, 2.3, shp))
    p = np.exp(rng.uniform(-2.3, 2.3, shp))
    cs = np.sqrt(gamma * p / rho)
    M = rng.uniform(0, 3, shp)
    d = rng.normal(size=(3,) + shp)
    d /= np.linalg.norm(d, axis=0)
    c.q0 = conserved3(gamma, rho, M * cs * d[0], M * cs * d[1], M * cs * d[2], p)
    c.name = f"rough3_{nx}x{ny}x{nz}"
    return c


def extrude(case2: "Case", nz: int, bc_z=(PERIODIC, PERIODIC)) -> Case3:
    """A 2-D case repeated along z (w = 0, unit dz): its 3-D solution is the
    2-D one in every z-slice.  Transported scalars ride along; Dirichlet z sides
    take the (rho, rho u, rho v, 0, rho E) of the west side and its scalars."""
    q = case2.q0
    ns = q.shape[0] - 4
    q3 = np.stack([q[0], q[1], q[2], np.zeros_like(q[0]), q[3]] + [q[4 + m] for m in range(ns)])
    q3 = np.ascontiguousarray(np.broadcast_to(q3[:, None], (5 + ns, nz) + q.shape[1:]))
    bcs = np.zeros((6, 5))
    for s in range(6):
        b = case2.bc_state[s if s < 4 else 0]
        bcs[s] = (b[0], b[1], b[2], 0.0, b[3])
    bsc = None
    if ns:
        bsc = np.zeros((6, ns))
        if case2.bc_scalar is not None:
            for s in range(6):
                bsc[s] = case2.bc_scalar[s if s < 4 else 0][:ns]
    return Case3(name=case2.name + f"_x{nz}", q0=q3, params=dict(case2.params),
                 bc=tuple(case2.bc) + tuple(bc_z), dx=case2.dx, dy=case2.dy, dz=1.0, bc_state=bcs,
                 nsteps=case2.nsteps, t_end=case2.t_end, bc_scalar=bsc)


def vortex3(n: int = 64, nz: int = 16, mach: float = 0.01, **params) -> Case3:
    """The low-Mach vortex of the second configuration extruded along z, with a
    seeded +-1e-6 checkerboard in all three directions and a small seeded w."""
    c2 = vortex(n, mach, checker_amp=0.0)
    c = extrude(c2, nz)
    gamma = c.params.get("gamma", 1.4)
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 500))
    rho = c.q0[0]
    u, v = c.q0[1] / rho, c.q0[2] / rho
    p = (gamma - 1.0) * (c.q0[4] - 0.5 * rho * (u * u + v * v))
    K, J, I = np.meshgrid(np.arange(nz), np.arange(n), np.arange(n), indexing="ij")
    p = p * (1.0 + 1e-6 * np.where((I + J + K) % 2 == 0, 1.0, -1.0) * rng.uniform(0.5, 1.5, p.shape))
    w = 0.1 * mach * np.sin(2 * math.pi * K / nz) * rng.uniform(0.5, 1.5, p.shape)
    c.q0 = conserved3(gamma, rho, u, v, w, p)
    c.dz = c.dx
    c.params.update(params)
    c.name = f"vortex3_{n}x{n}x{nz}_M{mach:g}"
    return c
