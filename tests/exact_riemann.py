"""Exact solution of the 1-D Euler Riemann problem for an ideal gas.

Textbook pressure-function method: the star pressure is the root of
f_L(p) + f_R(p) + (u_R - u_L) = 0, with the shock (Rankine-Hugoniot) branch for
p > p_K and the rarefaction (isentropic) branch otherwise; the solution is
then sampled along x/t.  Independent of the oracle; used to pin its shock-tube
results.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


def _fK(p, rho, pk, gamma):
    c = math.sqrt(gamma * pk / rho)
    if p > pk:
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        return (p - pk) * math.sqrt(A / (p + B))
    return 2.0 * c / (gamma - 1.0) * ((p / pk) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)


def star_state(left, right, gamma=1.4):
    """(p*, u*, rho*_L, rho*_R) for primitive states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    if 2.0 / (gamma - 1.0) * (cl + cr) <= ur - ul:
        raise ValueError("vacuum is generated")

    def fun(p):
        return _fK(p, rl, pl, gamma) + _fK(p, rr, pr, gamma) + (ur - ul)

    hi = max(pl, pr)
    while fun(hi) < 0.0:
        hi *= 2.0
    ps = brentq(fun, 1e-14, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    us = 0.5 * (ul + ur) + 0.5 * (_fK(ps, rr, pr, gamma) - _fK(ps, rl, pl, gamma))
    g1 = (gamma - 1.0) / (gamma + 1.0)

    def rho_star(rho, pk):
        if ps > pk:
            return rho * (ps / pk + g1) / (g1 * ps / pk + 1.0)
        return rho * (ps / pk) ** (1.0 / gamma)

    return ps, us, rho_star(rl, pl), rho_star(rr, pr)


def sample(left, right, x, x0, t, gamma=1.4):
    """Exact (rho, u, p) at positions x (array) and time t > 0."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us, rsl, rsr = star_state(left, right, gamma)
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    g = gamma
    out = np.zeros((3, len(x)))
    for m, xx in enumerate(x):
        s = (xx - x0) / t
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                out[:, m] = (rl, ul, pl) if s <= sl else (rsl, us, ps)
            else:  # left rarefaction
                csl = cl * (ps / pl) ** ((g - 1) / (2 * g))
                shl, stl = ul - cl, us - csl
                if s <= shl:
                    out[:, m] = (rl, ul, pl)
                elif s >= stl:
                    out[:, m] = (rsl, us, ps)
                else:
                    u = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    rho = rl * (c / cl) ** (2 / (g - 1))
                    out[:, m] = (rho, u, pl * (c / cl) ** (2 * g / (g - 1)))
        else:  # right of contact
            if ps > pr:
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                out[:, m] = (rr, ur, pr) if s >= sr else (rsr, us, ps)
            else:
                csr = cr * (ps / pr) ** ((g - 1) / (2 * g))
                shr, str_ = ur + cr, us + csr
                if s >= shr:
                    out[:, m] = (rr, ur, pr)
                elif s <= str_:
                    out[:, m] = (rsr, us, ps)
                else:
                    u = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    rho = rr * (c / cr) ** (2 / (g - 1))
                    out[:, m] = (rho, u, pr * (c / cr) ** (2 * g / (g - 1)))
    return out
