"""FP64 CPU oracle of the Roe-AM solver (arXiv 1711.09272) -- TEST INFRASTRUCTURE ONLY.

Python wrapper (ctypes) around ``roeam_oracle.c``.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import this package.  It
shares no code with the GPU library; the only common input is the seeded
generator module ``workloads``.

Parity unpinned (documented readings, checked only oracle == GPU): the
modified entropy fix / rotated Riemann solver term of Eq. (86), the weight of
the expansion-shock fix of Eq. (92), MUSCL-minmod, the slip-wall ghost rule
and the time-step rule.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "roeam_oracle.c")
_SRC3 = os.path.join(_HERE, "roeam_oracle3d.c")
_LIB = os.path.join(_HERE, "libroeam_oracle.so")

V_XI_UNGATED = 1 << 0
V_EXPFIX_F8 = 1 << 1
V_CLAMP_UPRIME = 1 << 2
V_NO_EQ92 = 1 << 3
V_XI_ROE = 1 << 4
V_DUP_ROE = 1 << 5
V_XI_EQ46 = 1 << 6
V_DUP_ZERO = 1 << 7

SCHEME_ROEAM, SCHEME_ROE, SCHEME_ROE_HARTEN = 0, 1, 2
BC_DIRICHLET = 3
BC_SLIPWALL = 2
BC_MOVING = 4  # a side split at a + b t: its lo kind below, its hi kind above
MAX_SCALARS = 2  # transported scalars (rho k rows of Eq. 85) a grid may carry


def _stale() -> bool:
    if not os.path.exists(_LIB):
        return True
    t = os.path.getmtime(_LIB)
    return any(os.path.getmtime(f) > t for f in (_SRC, _SRC3, os.path.join(_HERE, "roeam_oracle.h")))


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, no fused multiply-add contraction)."""
    if force or _stale():
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-o", _LIB, _SRC, _SRC3, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("mach_ref", ctypes.c_double),
                ("u_ref", ctypes.c_double), ("eps1", ctypes.c_double), ("eps2", ctypes.c_double),
                ("eps_lambda", ctypes.c_double), ("s1_mode", ctypes.c_int), ("order", ctypes.c_int),
                ("time_scheme", ctypes.c_int), ("scheme", ctypes.c_int), ("variant", ctypes.c_uint)]


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("metric", ctypes.c_int),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("xn", ctypes.POINTER(ctypes.c_double)), ("yn", ctypes.POINTER(ctypes.c_double)),
                ("bc", ctypes.c_int * 4), ("bc_state", (ctypes.c_double * 4) * 4),
                ("nscalars", ctypes.c_int), ("bc_scalar", (ctypes.c_double * MAX_SCALARS) * 4),
                ("split_a", ctypes.c_double * 4), ("split_b", ctypes.c_double * 4), ("split_hi", ctypes.c_int * 4),
                ("bc_state_hi", (ctypes.c_double * 4) * 4), ("t_bc", ctypes.c_double),
                ("split_lo", ctypes.c_int * 4)]


_DIAG_FIELDS = ["UL", "UR", "U", "dU", "dp", "rho", "u", "v", "H", "c", "M", "Mbar", "theta",
                "ct", "Ut", "absUp", "s1", "fef", "frr", "xi", "dpp", "dpu", "dUp", "dUuR", "dUuL"]


class _Diag(ctypes.Structure):
    _fields_ = [(f, ctypes.c_double) for f in _DIAG_FIELDS]


class _Stats(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("dt_last", ctypes.c_double), ("max_rate", ctypes.c_double),
                ("steps", ctypes.c_long), ("nonphys", ctypes.c_int), ("neg_uprime_faces", ctypes.c_long)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _stale():
            build(force=True)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_f.restype = ctypes.c_double
        L.orc_f.argtypes = [ctypes.c_double]
        L.orc_detector_P.restype = ctypes.c_double
        L.orc_detector_P.argtypes = [ctypes.c_double] * 4
        L.orc_face_flux.restype = None
        L.orc_face_flux.argtypes = [ctypes.POINTER(_Params), dp, dp, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, dp, ctypes.POINTER(_Diag)]
        L.orc_face_flux_sc.restype = None
        L.orc_face_flux_sc.argtypes = [ctypes.POINTER(_Params), dp, dp, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int, dp]
        L.orc_physical_flux.restype = None
        L.orc_physical_flux.argtypes = [ctypes.c_double, dp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_residual.restype = ctypes.c_int
        L.orc_residual.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Grid), dp, dp, dp]
        L.orc_rotated_mach.restype = ctypes.c_int
        L.orc_rotated_mach.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Grid), dp, dp, dp]
        L.orc_max_rate.restype = ctypes.c_int
        L.orc_max_rate.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Grid), dp, dp]
        L.orc_run.restype = ctypes.c_int
        L.orc_run.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Grid), dp, ctypes.c_long,
                              ctypes.c_double, ctypes.POINTER(_Stats)]
        L.orc_cell_areas.restype = None
        L.orc_cell_areas.argtypes = [ctypes.POINTER(_Grid), dp]
        L.orc3_physical_flux.restype = None
        L.orc3_physical_flux.argtypes = [ctypes.c_double, dp, dp, dp]
        L.orc3_face_flux.restype = None
        L.orc3_face_flux.argtypes = [ctypes.POINTER(_Params), dp, dp, dp, ctypes.c_double, dp]
        L.orc3_face_flux_sc.restype = None
        L.orc3_face_flux_sc.argtypes = [ctypes.POINTER(_Params), dp, dp, dp, ctypes.c_double, ctypes.c_int, dp]
        L.orc3_residual.restype = ctypes.c_int
        L.orc3_residual.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Grid3), dp, dp, dp]
        L.orc3_max_rate.restype = ctypes.c_int
        L.orc3_max_rate.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Grid3), dp, dp]
        L.orc3_run.restype = ctypes.c_int
        L.orc3_run.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Grid3), dp, ctypes.c_long,
                               ctypes.c_double, ctypes.POINTER(_Stats)]
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_max_threads.argtypes = []
        _lib = L
    return _lib


def set_threads(n: int):
    """Threads of the oracle's row loops (OpenMP); results are the same bits for any count."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(p: Dict) -> _Params:
    return _Params(p.get("gamma", 1.4), p.get("cfl", 0.4), p.get("mach_ref", 1.0), p.get("u_ref", 1.0),
                   p.get("eps1", 0.0), p.get("eps2", 0.05), p.get("eps_lambda", 0.1),
                   int(p.get("s1_mode", 0)), int(p.get("order", 1)), int(p.get("time_scheme", 0)),
                   int(p.get("scheme", 0)), int(p.get("variant", 0)))


class GridSpec:
    """Holds the ctypes grid and keeps the node arrays alive."""

    def __init__(self, case):
        self.nx, self.ny = case.nx, case.ny
        self._keep = []
        g = _Grid()
        g.nx, g.ny = case.nx, case.ny
        g.metric = case.metric
        g.dx, g.dy = case.dx, case.dy
        if case.metric == 1:
            xn = np.ascontiguousarray(case.xn, dtype=np.float64)
            yn = np.ascontiguousarray(case.yn, dtype=np.float64)
            assert xn.shape == (case.ny + 1, case.nx + 1)
            self._keep += [xn, yn]
            g.xn, g.yn = _dptr(xn), _dptr(yn)
        for s in range(4):
            g.bc[s] = int(case.bc[s])
            for k in range(4):
                g.bc_state[s][k] = float(case.bc_state[s][k])
        ns = case.q0.shape[0] - 4
        assert 0 <= ns <= MAX_SCALARS
        g.nscalars = ns
        bcs = getattr(case, "bc_scalar", None)
        if ns and bcs is not None:
            for s in range(4):
                for m in range(ns):
                    g.bc_scalar[s][m] = float(bcs[s][m])
        # moving-split sides: {side: (a, b, hi_kind, state_hi[, lo_kind])}; below the split the
        # lo kind (default Dirichlet: the side's bc_state), above it the hi kind
        for side, spec in (getattr(case, "moving", None) or {}).items():
            sa, sb, hi, st_hi = spec[:4]
            lo = spec[4] if len(spec) > 4 else BC_DIRICHLET
            g.split_a[side], g.split_b[side], g.split_hi[side], g.split_lo[side] = float(sa), float(sb), int(hi), int(lo)
            for k in range(4):
                g.bc_state_hi[side][k] = float(st_hi[k]) if st_hi is not None else 0.0
        g.t_bc = float(getattr(case, "t_bc", 0.0))
        self.g = g


def f(phi: float) -> float:
    return lib().orc_f(float(phi))


def detector_P(pA, rhoA, pB, rhoB) -> float:
    return lib().orc_detector_P(float(pA), float(rhoA), float(pB), float(rhoB))


def physical_flux(W, nx, ny, gamma=1.4) -> np.ndarray:
    W = np.ascontiguousarray(W, dtype=np.float64)
    F = np.zeros(4)
    lib().orc_physical_flux(gamma, _dptr(W), float(nx), float(ny), _dptr(F))
    return F


def face_flux(params: Dict, WL, WR, nx: float, ny: float, s1: float = 1.0) -> Tuple[np.ndarray, Dict]:
    """Numerical flux per unit face length for one face, plus every intermediate."""
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    F = np.zeros(4)
    d = _Diag()
    prm = make_params(params)
    lib().orc_face_flux(ctypes.byref(prm), _dptr(WL), _dptr(WR), float(nx), float(ny), float(s1),
                        _dptr(F), ctypes.byref(d))
    return F, {k: getattr(d, k) for k in _DIAG_FIELDS}


def face_flux_sc(params: Dict, WL, WR, nx: float, ny: float, s1: float = 1.0) -> np.ndarray:
    """Flux per unit face length with transported scalars: W = (rho, u, v, p, k_1, ..)."""
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    ns = len(WL) - 4
    F = np.zeros(4 + ns)
    prm = make_params(params)
    lib().orc_face_flux_sc(ctypes.byref(prm), _dptr(WL), _dptr(WR), float(nx), float(ny), float(s1), ns, _dptr(F))
    return F


class NonPhysical(RuntimeError):
    pass


def _check(rc: int):
    if rc == -4:
        raise NonPhysical("non-physical state (rho <= 0, p <= 0 or non-finite)")
    if rc != 0:
        raise RuntimeError(f"oracle error {rc}")


def residual(case, q: Optional[np.ndarray] = None, params: Optional[Dict] = None,
             with_scale: bool = False):
    """R = dQ/dt for the case's grid; q defaults to case.q0.  Returns r (and the
    per-cell flux scale sum_faces |F| |S| / Omega when ``with_scale``)."""
    q = np.ascontiguousarray(case.q0 if q is None else q, dtype=np.float64)
    assert q.shape == (case.q0.shape[0], case.ny, case.nx)
    gs = GridSpec(case)
    prm = make_params(params or case.params)
    r = np.zeros_like(q)
    sc = np.zeros_like(q) if with_scale else None
    rc = lib().orc_residual(ctypes.byref(prm), ctypes.byref(gs.g), _dptr(q), _dptr(r),
                            _dptr(sc) if with_scale else None)
    _check(rc)
    return (r, sc) if with_scale else r


def rotated_mach(case, q: Optional[np.ndarray] = None, params: Optional[Dict] = None):
    """f_rr / c on the i-faces [ny, nx+1] and the j-faces [ny+1, nx] (Fig. 7's diagnostic)."""
    q = np.ascontiguousarray(case.q0 if q is None else q, dtype=np.float64)
    gs = GridSpec(case)
    prm = make_params(params or case.params)
    fx = np.zeros((case.ny, case.nx + 1))
    fy = np.zeros((case.ny + 1, case.nx))
    _check(lib().orc_rotated_mach(ctypes.byref(prm), ctypes.byref(gs.g), _dptr(q), _dptr(fx), _dptr(fy)))
    return fx, fy


def max_rate(case, q: Optional[np.ndarray] = None, params: Optional[Dict] = None) -> float:
    q = np.ascontiguousarray(case.q0 if q is None else q, dtype=np.float64)
    gs = GridSpec(case)
    prm = make_params(params or case.params)
    out = ctypes.c_double(0.0)
    _check(lib().orc_max_rate(ctypes.byref(prm), ctypes.byref(gs.g), _dptr(q), ctypes.byref(out)))
    return out.value


def run(case, nsteps: Optional[int] = None, t_end: Optional[float] = None,
        q: Optional[np.ndarray] = None, params: Optional[Dict] = None, t0: float = 0.0,
        raise_on_nonphys: bool = True):
    """Advance a copy of the state; returns (q, stats dict)."""
    q = np.array(case.q0 if q is None else q, dtype=np.float64, order="C", copy=True)
    gs = GridSpec(case)
    prm = make_params(params or case.params)
    st = _Stats()
    st.t = t0
    rc = lib().orc_run(ctypes.byref(prm), ctypes.byref(gs.g), _dptr(q),
                       int(case.nsteps if nsteps is None else nsteps),
                       float(case.t_end if t_end is None else t_end), ctypes.byref(st))
    stats = {k: getattr(st, k) for k, _ in _Stats._fields_}
    if rc == -4 and not raise_on_nonphys:
        return q, stats
    _check(rc)
    return q, stats


def cell_areas(case) -> np.ndarray:
    gs = GridSpec(case)
    om = np.zeros((case.ny, case.nx))
    lib().orc_cell_areas(ctypes.byref(gs.g), _dptr(om))
    return om


# --------------------------------------------------------------------------
# 3-D (uniform Cartesian grids)
# --------------------------------------------------------------------------

class _Grid3(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("dx", ctypes.c_double),
                ("dy", ctypes.c_double), ("dz", ctypes.c_double), ("bc", ctypes.c_int * 6),
                ("bc_state", (ctypes.c_double * 5) * 6), ("nscalars", ctypes.c_int),
                ("bc_scalar", (ctypes.c_double * MAX_SCALARS) * 6)]


def _grid3(case) -> _Grid3:
    g = _Grid3()
    g.nx, g.ny, g.nz = case.nx, case.ny, case.nz
    g.dx, g.dy, g.dz = case.dx, case.dy, case.dz
    for s in range(6):
        g.bc[s] = int(case.bc[s])
        for k in range(5):
            g.bc_state[s][k] = float(case.bc_state[s][k])
    ns = case.q0.shape[0] - 5
    assert 0 <= ns <= MAX_SCALARS
    g.nscalars = ns
    bcs = getattr(case, "bc_scalar", None)
    if ns and bcs is not None:
        for s in range(6):
            for m in range(ns):
                g.bc_scalar[s][m] = float(bcs[s][m])
    return g


def physical_flux3(W, n, gamma: float = 1.4) -> np.ndarray:
    W = np.ascontiguousarray(W, dtype=np.float64)
    nv = np.ascontiguousarray(n, dtype=np.float64)
    F = np.zeros(5)
    lib().orc3_physical_flux(float(gamma), _dptr(W), _dptr(nv), _dptr(F))
    return F


def face_flux3(params: Dict, WL, WR, n, s1: float = 1.0) -> np.ndarray:
    """3-D numerical flux per unit face area; W = (rho, u, v, w, p), n unit."""
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    nv = np.ascontiguousarray(n, dtype=np.float64)
    F = np.zeros(5)
    prm = make_params(params)
    lib().orc3_face_flux(ctypes.byref(prm), _dptr(WL), _dptr(WR), _dptr(nv), float(s1), _dptr(F))
    return F


def face_flux3_sc(params: Dict, WL, WR, n, s1: float = 1.0) -> np.ndarray:
    """3-D flux with transported scalars: W = (rho, u, v, w, p, k_1, ..), F has len(W) rows."""
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    ns = WL.shape[0] - 5
    assert WR.shape == WL.shape and 0 <= ns <= MAX_SCALARS
    nv = np.ascontiguousarray(n, dtype=np.float64)
    F = np.zeros(5 + ns)
    prm = make_params(params)
    lib().orc3_face_flux_sc(ctypes.byref(prm), _dptr(WL), _dptr(WR), _dptr(nv), float(s1), ns, _dptr(F))
    return F


def residual3(case, q: Optional[np.ndarray] = None, params: Optional[Dict] = None, with_scale: bool = False):
    q = np.ascontiguousarray(case.q0 if q is None else q, dtype=np.float64)
    assert q.shape == (case.q0.shape[0], case.nz, case.ny, case.nx)
    g = _grid3(case)
    prm = make_params(params or case.params)
    r = np.zeros_like(q)
    sc = np.zeros_like(q) if with_scale else None
    _check(lib().orc3_residual(ctypes.byref(prm), ctypes.byref(g), _dptr(q), _dptr(r),
                               _dptr(sc) if with_scale else None))
    return (r, sc) if with_scale else r


def max_rate3(case, q: Optional[np.ndarray] = None, params: Optional[Dict] = None) -> float:
    q = np.ascontiguousarray(case.q0 if q is None else q, dtype=np.float64)
    g = _grid3(case)
    prm = make_params(params or case.params)
    out = ctypes.c_double(0.0)
    _check(lib().orc3_max_rate(ctypes.byref(prm), ctypes.byref(g), _dptr(q), ctypes.byref(out)))
    return out.value


def run3(case, nsteps: Optional[int] = None, t_end: Optional[float] = None, q: Optional[np.ndarray] = None,
         params: Optional[Dict] = None, t0: float = 0.0):
    q = np.array(case.q0 if q is None else q, dtype=np.float64, order="C", copy=True)
    g = _grid3(case)
    prm = make_params(params or case.params)
    st = _Stats()
    st.t = t0
    rc = lib().orc3_run(ctypes.byref(prm), ctypes.byref(g), _dptr(q), int(case.nsteps if nsteps is None else nsteps),
                        float(case.t_end if t_end is None else t_end), ctypes.byref(st))
    _check(rc)
    return q, {k: getattr(st, k) for k, _ in _Stats._fields_}
