"""Python binding of the gfx950 Roe-AM library (``libroeam.so``, C ABI in include/roeam.h).

Argument marshalling only: every step of the residual and time step runs in
the library's HIP kernels.  PyTorch supplies device memory and streams.  The
library must be built (``python -m paper_1711_09272_amd.build``); importing
the binding without it raises ImportError -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libroeam.so")

OK, EINVAL, ENOMEM, EDEVICE, ENONPHYS, EBUSY, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
MAX_SCALARS = 2  # transported scalars (rho k rows) a grid may carry
BC_PERIODIC, BC_TRANSMISSIVE, BC_SLIPWALL, BC_DIRICHLET, BC_MOVING = 0, 1, 2, 3, 4
V_XI_UNGATED, V_EXPFIX_F8, V_CLAMP_UPRIME = 1, 2, 4
# stage-kernel tile shapes: cells x cells / threads per workgroup
SHAPES = ["32x15/256", "16x15/128", "8x7/64", "8x7/128", "16x15/512", "32x7/512", "16x15/256", "32x7/256", "16x7/256"]

EXPORTS = [
    "roeam_ctx_create", "roeam_ctx_destroy", "roeam_ctx_set_stream", "roeam_last_error",
    "roeam_grid_create", "roeam_grid_destroy", "roeam_grid_layout", "roeam_grid_set_tile_shape",
    "roeam_grid_tile_shape", "roeam_grid_set_scalars", "roeam_grid_set_moving_side", "roeam_grid_set_boundary_time",
    "roeam_residual", "roeam_step",
    "roeam_last_stats", "roeam_profile_step", "roeam_batch_reserve", "roeam_batch_footprint", "roeam_batch_submit",
    "roeam_batch_run", "roeam_batch_profile_run", "roeam_batch_poll", "roeam_batch_attach", "roeam_residual_norms",
    "roeam_residual_norms3d", "roeam_residual_norms_noalloc", "roeam_batch_configure", "roeam_batch_info",
    "roeam_grid3d_create", "roeam_grid3d_destroy", "roeam_grid3d_layout", "roeam_grid3d_set_tile_shape",
    "roeam_grid3d_tile_shape",
    "roeam_grid3d_set_scalars", "roeam_residual3d", "roeam_step3d", "roeam_last_stats3d",
]
# 3-D stage-kernel brick shapes: cells x cells x cells / threads per workgroup
SHAPES3 = ["8x8x4/256", "8x4x4/128", "16x8x4/512", "16x4x4/256", "8x8x4/320", "8x4x4/192", "16x8x4/640",
           "8x8x8/576", "16x8x4/512p", "8x8x8/512p",  # p: persistent, prefetching the next brick's halo
           # z: z-marching column tiles TX x TY walking runs of TZ planes (z*: one round of workgroups,
           # each tile's height cut into balanced runs)
           "16x15z4/256", "16x15z8/256", "16x15z16/256", "16x15z*/256"]


class RoeamError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"roeam error {code}: {msg}")
        self.code = code


class NonPhysicalError(RoeamError):
    pass


class Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("mach_ref", ctypes.c_double),
                ("u_ref", ctypes.c_double), ("eps1", ctypes.c_double), ("eps2", ctypes.c_double),
                ("s1_mode", ctypes.c_int), ("order", ctypes.c_int), ("time_scheme", ctypes.c_int),
                ("precision", ctypes.c_int), ("variant", ctypes.c_uint), ("scheme", ctypes.c_int),
                ("eps_lambda", ctypes.c_double)]


class Metrics(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("xn", ctypes.POINTER(ctypes.c_double)), ("yn", ctypes.POINTER(ctypes.c_double))]


class StepStats(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("dt_last", ctypes.c_double), ("max_rate", ctypes.c_double),
                ("steps", ctypes.c_long), ("nonphys", ctypes.c_int)]

    def as_dict(self) -> Dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchStats(ctypes.Structure):
    _fields_ = [("captures", ctypes.c_long), ("graph_launches", ctypes.c_long), ("iterations", ctypes.c_long),
                ("tunes", ctypes.c_long), ("resident", ctypes.c_int), ("queued", ctypes.c_int),
                ("graph_iters", ctypes.c_int), ("persistent", ctypes.c_int), ("policy", ctypes.c_int),
                ("shape", ctypes.c_int), ("max_resident", ctypes.c_int)]


ADMIT_FIFO, ADMIT_SHORTEST = 0, 1


class SolveDesc(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_void_p), ("params", Params), ("q0", ctypes.c_void_p),
                ("q0_on_device", ctypes.c_int), ("nsteps", ctypes.c_long), ("t_end", ctypes.c_double),
                ("q_out", ctypes.c_void_p), ("q_out_on_device", ctypes.c_int)]


_lib = None


def lib():
    """Load libroeam.so (raises ImportError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1711_09272_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "roeam_ctx_create": (i, [i, vp, ctypes.POINTER(vp)]),
        "roeam_ctx_destroy": (i, [vp]),
        "roeam_ctx_set_stream": (i, [vp, vp]),
        "roeam_last_error": (ctypes.c_char_p, [vp]),
        "roeam_grid_create": (i, [vp, i, i, ctypes.POINTER(Metrics), ctypes.POINTER(ctypes.c_int * 4), vp,
                                  ctypes.POINTER(vp)]),
        "roeam_grid_destroy": (i, [vp]),
        "roeam_grid_layout": (i, [vp, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(ctypes.c_long)]),
        "roeam_grid_set_tile_shape": (i, [vp, i]),
        "roeam_grid_tile_shape": (i, [vp, ctypes.POINTER(Params), ctypes.POINTER(i)]),
        "roeam_grid_set_scalars": (i, [vp, i, vp]),
        "roeam_grid_set_moving_side": (i, [vp, i, d, d, i, i, vp]),
        "roeam_grid_set_boundary_time": (i, [vp, d]),
        "roeam_residual": (i, [vp, vp, ctypes.POINTER(Params), vp, vp, vp]),
        "roeam_step": (i, [vp, vp, ctypes.POINTER(Params), vp, ctypes.c_long, d, d, ctypes.POINTER(StepStats)]),
        "roeam_last_stats": (i, [vp, vp, ctypes.POINTER(StepStats)]),
        "roeam_residual_norms": (i, [vp, vp, vp, vp]),
        "roeam_residual_norms3d": (i, [vp, vp, vp, vp]),
        "roeam_residual_norms_noalloc": (i, [vp, vp, vp, vp]),
        "roeam_profile_step": (i, [vp, vp, ctypes.POINTER(Params), vp, ctypes.c_long, d,
                                   ctypes.POINTER(ctypes.c_double * 4), ctypes.POINTER(ctypes.c_long)]),
        "roeam_batch_reserve": (i, [vp, ctypes.c_size_t]),
        "roeam_batch_attach": (i, [vp, vp, ctypes.c_size_t]),
        "roeam_batch_footprint": (ctypes.c_size_t, [vp]),
        "roeam_batch_submit": (i, [vp, i, ctypes.POINTER(SolveDesc), ctypes.POINTER(ctypes.c_uint64)]),
        "roeam_batch_run": (i, [vp, ctypes.c_long, ctypes.POINTER(i)]),
        "roeam_batch_profile_run": (i, [vp, ctypes.c_long, ctypes.POINTER(i), ctypes.POINTER(ctypes.c_double * 4),
                                        ctypes.POINTER(ctypes.c_long)]),
        "roeam_batch_poll": (i, [vp, ctypes.c_uint64, ctypes.POINTER(i), ctypes.POINTER(StepStats)]),
        "roeam_batch_configure": (i, [vp, i, i, i, i, i]),
        "roeam_batch_info": (i, [vp, ctypes.POINTER(BatchStats)]),
        "roeam_grid3d_create": (i, [vp, i, i, i, d, d, d, ctypes.POINTER(ctypes.c_int * 6), vp, ctypes.POINTER(vp)]),
        "roeam_grid3d_destroy": (i, [vp]),
        "roeam_grid3d_layout": (i, [vp, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i),
                                    ctypes.POINTER(ctypes.c_long)]),
        "roeam_grid3d_set_tile_shape": (i, [vp, i]),
        "roeam_grid3d_tile_shape": (i, [vp, i, ctypes.POINTER(i)]),
        "roeam_grid3d_set_scalars": (i, [vp, i, vp]),
        "roeam_residual3d": (i, [vp, vp, ctypes.POINTER(Params), vp, vp, vp]),
        "roeam_step3d": (i, [vp, vp, ctypes.POINTER(Params), vp, ctypes.c_long, d, d, ctypes.POINTER(StepStats)]),
        "roeam_last_stats3d": (i, [vp, vp, ctypes.POINTER(StepStats)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def params(d: Dict) -> Params:
    """Params from a dict with the keys of workloads.default_params."""
    return Params(float(d.get("gamma", 1.4)), float(d.get("cfl", 0.4)), float(d.get("mach_ref", 1.0)),
                  float(d.get("u_ref", 1.0)), float(d.get("eps1", 0.0)), float(d.get("eps2", 0.05)),
                  int(d.get("s1_mode", 0)), int(d.get("order", 1)), int(d.get("time_scheme", 0)),
                  int(d.get("precision", 0)), int(d.get("variant", 0)), int(d.get("scheme", 0)),
                  float(d.get("eps_lambda", 0.1)))


def _stream_ptr(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class Context:
    """A library context on one device.

    The library enqueues on its own non-null torch stream (the null stream
    cannot be captured into HIP graphs).  Every call below first makes that
    stream wait for the caller's current torch stream and afterwards makes the
    current stream wait for it, so library calls are ordered with the caller's
    torch work exactly as if they ran on the current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.device = device
        torch.cuda.set_device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        h = ctypes.c_void_p()
        rc = lib().roeam_ctx_create(device, ctypes.c_void_p(_stream_ptr(self.stream)), ctypes.byref(h))
        if rc != OK:
            raise RoeamError(rc, "context creation failed")
        self.h = h

    def enter(self):
        import torch
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def leave(self):
        import torch
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def check(self, rc: int):
        if rc == OK:
            return
        msg = lib().roeam_last_error(self.h).decode()
        if rc == ENONPHYS:
            raise NonPhysicalError(rc, msg)
        raise RoeamError(rc, msg)

    def set_stream(self, stream):
        self.check(lib().roeam_ctx_set_stream(self.h, ctypes.c_void_p(_stream_ptr(stream))))
        self.stream = stream

    def close(self):
        if getattr(self, "h", None):
            lib().roeam_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Grid:
    """An immutable structured grid of the library (sizes, metrics, boundary kinds)."""

    def __init__(self, ctx: Context, nx: int, ny: int, dx: float = None, dy: float = None,
                 xn: Optional[np.ndarray] = None, yn: Optional[np.ndarray] = None,
                 bc: Sequence[int] = (0, 0, 0, 0), bc_state: Optional[np.ndarray] = None):
        self.ctx = ctx
        m = Metrics()
        self._keep = []
        if xn is None:
            m.kind, m.dx, m.dy = 0, float(dx), float(dy)
        else:
            xa = np.ascontiguousarray(xn, dtype=np.float64)
            ya = np.ascontiguousarray(yn, dtype=np.float64)
            assert xa.shape == (ny + 1, nx + 1) and ya.shape == (ny + 1, nx + 1)
            self._keep += [xa, ya]
            m.kind = 1
            m.xn = xa.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            m.yn = ya.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        bca = (ctypes.c_int * 4)(*[int(b) for b in bc])
        st = None
        if bc_state is not None:
            sa = np.ascontiguousarray(bc_state, dtype=np.float64).reshape(16)
            self._keep.append(sa)
            st = ctypes.c_void_p(sa.ctypes.data)
        h = ctypes.c_void_p()
        ctx.check(lib().roeam_grid_create(ctx.h, int(nx), int(ny), ctypes.byref(m), ctypes.byref(bca), st,
                                          ctypes.byref(h)))
        self.h = h
        a, b, p = ctypes.c_int(), ctypes.c_int(), ctypes.c_long()
        lib().roeam_grid_layout(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(p))
        self.nx, self.ny, self.pitch = a.value, b.value, p.value
        self.nsc = 0

    @classmethod
    def from_case(cls, ctx: Context, case) -> "Grid":
        g = cls(ctx, case.nx, case.ny, dx=case.dx, dy=case.dy, xn=case.xn, yn=case.yn, bc=case.bc,
                bc_state=case.bc_state)
        ns = case.q0.shape[0] - 4
        if ns:
            g.set_scalars(ns, getattr(case, "bc_scalar", None))
        for side, spec in (getattr(case, "moving", None) or {}).items():
            a, b, hi, state_hi = spec[:4]
            g.set_moving_side(side, a, b, hi, state_hi, lo_kind=spec[4] if len(spec) > 4 else BC_DIRICHLET)
        g.set_boundary_time(getattr(case, "t_bc", 0.0))
        return g

    def set_moving_side(self, side: int, a: float, b: float, hi_kind: int, state_hi=None, lo_kind: int = BC_DIRICHLET):
        """Split a + b t of a BC_MOVING side; below it the side's Dirichlet state or a slip wall
        (lo_kind), above it a slip wall or the conserved state_hi (hi_kind)."""
        arg = None
        if state_hi is not None:
            sa = np.ascontiguousarray(state_hi, dtype=np.float64).reshape(4)
            self._keep.append(sa)
            arg = ctypes.c_void_p(sa.ctypes.data)
        self.ctx.check(lib().roeam_grid_set_moving_side(self.h, int(side), float(a), float(b), int(lo_kind),
                                                        int(hi_kind), arg))

    def set_boundary_time(self, t: float):
        """Time at which residual() evaluates moving sides."""
        self.ctx.check(lib().roeam_grid_set_boundary_time(self.h, float(t)))

    def set_scalars(self, nscalars: int, bc_scalar: Optional[np.ndarray] = None):
        """Carry nscalars transported scalars (state rows 4..); bc_scalar: [4 sides, nscalars]
        Dirichlet rho k_m."""
        arg = None
        if bc_scalar is not None and nscalars:
            sa = np.ascontiguousarray(np.asarray(bc_scalar, dtype=np.float64)[:, :nscalars]).reshape(-1)
            self._keep.append(sa)
            arg = ctypes.c_void_p(sa.ctypes.data)
        self.ctx.check(lib().roeam_grid_set_scalars(self.h, int(nscalars), arg))
        self.nsc = int(nscalars)

    @property
    def rows(self) -> int:
        return 4 + self.nsc

    def empty_state(self):
        import torch
        return torch.zeros((self.rows, self.ny, self.pitch), dtype=torch.float64, device=f"cuda:{self.ctx.device}")

    def to_device(self, q: np.ndarray):
        import torch
        t = self.empty_state()
        t[:, :, : self.nx] = torch.from_numpy(np.ascontiguousarray(q, dtype=np.float64))
        return t

    def from_device(self, t) -> np.ndarray:
        return t[:, :, : self.nx].detach().cpu().numpy().copy()

    def set_tile_shape(self, shape: int):
        """Tile shape (see SHAPES); -1 = autotune."""
        self.ctx.check(lib().roeam_grid_set_tile_shape(self.h, int(shape)))

    def tile_shape(self, prm: Dict) -> int:
        out = ctypes.c_int()
        p = params(prm)
        self.ctx.check(lib().roeam_grid_tile_shape(self.h, ctypes.byref(p), ctypes.byref(out)))
        return out.value

    def footprint(self) -> int:
        return int(lib().roeam_batch_footprint(self.h))

    def close(self):
        if getattr(self, "h", None):
            lib().roeam_grid_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dev_ptr(t, grid: Grid) -> ctypes.c_void_p:
    import torch
    assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
    assert tuple(t.shape) == (grid.rows, grid.ny, grid.pitch), (tuple(t.shape), (grid.rows, grid.ny, grid.pitch))
    return ctypes.c_void_p(t.data_ptr())


def residual(ctx: Context, grid: Grid, prm: Dict, q, r=None, rate_out=None):
    """R = dQ/dt of state tensor q (device, [4, ny, pitch]); returns r.
    rate_out: optional 1-element float64 device tensor for the max explicit rate."""
    if r is None:
        r = grid.empty_state()
    p = params(prm)
    rp = ctypes.c_void_p(rate_out.data_ptr()) if rate_out is not None else None
    ctx.enter()
    try:
        ctx.check(lib().roeam_residual(ctx.h, grid.h, ctypes.byref(p), _dev_ptr(q, grid), _dev_ptr(r, grid), rp))
    finally:
        ctx.leave()
    return r


def step(ctx: Context, grid: Grid, prm: Dict, q, nsteps: int, t0: float = 0.0, t_end: float = 0.0,
         sync: bool = True) -> Optional[Dict]:
    """Advance q in place; returns the step statistics when sync (else None)."""
    p = params(prm)
    st = StepStats()
    ctx.enter()
    try:
        ctx.check(lib().roeam_step(ctx.h, grid.h, ctypes.byref(p), _dev_ptr(q, grid), int(nsteps), float(t0),
                                   float(t_end), ctypes.byref(st) if sync else None))
    finally:
        ctx.leave()
    return st.as_dict() if sync else None


def residual_norms(ctx: Context, grid, r):
    """RMS and max |.| per row of a residual tensor (2-D or 3-D grid); returns a
    float64 device tensor [2, rows] (row 0: RMS, row 1: max)."""
    import torch
    three_d = isinstance(grid, Grid3)
    rows = grid.rows
    out = torch.zeros(2 * rows, dtype=torch.float64, device=f"cuda:{ctx.device}")
    rp = _dev_ptr3(r, grid) if three_d else _dev_ptr(r, grid)
    fn = lib().roeam_residual_norms3d if three_d else lib().roeam_residual_norms
    ctx.enter()
    try:
        ctx.check(fn(ctx.h, grid.h, rp, ctypes.c_void_p(out.data_ptr())))
    finally:
        ctx.leave()
    return out.view(2, rows)


def residual_norms_noalloc(ctx: Context, grid: Grid, r, out):
    """roeam_residual_norms_noalloc: the norms of a 2-D residual tensor into the
    caller's float64 device tensor `out` (2 * rows elements); nothing is
    allocated, here or in the library.  Returns `out` viewed as [2, rows]."""
    rows = grid.rows
    if out.dtype != __import__("torch").float64 or not out.is_cuda or out.numel() != 2 * rows \
            or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous float64 device tensor of {2 * rows} elements")
    ctx.enter()
    try:
        ctx.check(lib().roeam_residual_norms_noalloc(ctx.h, grid.h, _dev_ptr(r, grid), ctypes.c_void_p(out.data_ptr())))
    finally:
        ctx.leave()
    return out.view(2, rows)


def last_stats(ctx: Context, grid: Grid) -> Dict:
    st = StepStats()
    ctx.check(lib().roeam_last_stats(ctx.h, grid.h, ctypes.byref(st)))
    ctx.leave()
    return st.as_dict()


def profile_step(ctx: Context, grid: Grid, prm: Dict, q, nsteps: int, t0: float = 0.0):
    """Advance q by nsteps steps with HIP events around every stage kernel; returns
    (mean ms of the first to fourth stage kernels of a step, number of timed launches)."""
    p = params(prm)
    out = (ctypes.c_double * 4)()
    n = ctypes.c_long()
    ctx.enter()
    try:
        ctx.check(lib().roeam_profile_step(ctx.h, grid.h, ctypes.byref(p), _dev_ptr(q, grid), int(nsteps),
                                           float(t0), ctypes.byref(out), ctypes.byref(n)))
    finally:
        ctx.leave()
    return list(out), n.value


# ---------------------------------------------------------------------------
# batched and served solves
# ---------------------------------------------------------------------------

class Solve:
    """One batched solve: grid, parameters, initial state, run length and output.

    q0 / q_out: numpy arrays (host) or torch tensors (device) of shape
    [grid.rows, ny, pitch]; they must stay alive until the ticket reports done."""

    def __init__(self, grid: Grid, prm: Dict, q0, nsteps: int, t_end: float = 0.0, q_out=None):
        self.grid, self.prm, self.nsteps, self.t_end = grid, prm, int(nsteps), float(t_end)
        self.q0 = q0
        if q_out is None:
            q_out = np.zeros((grid.rows, grid.ny, grid.pitch))
        self.q_out = q_out
        self.ticket = None

    @staticmethod
    def _ptr(a, grid):
        if isinstance(a, np.ndarray):
            assert a.dtype == np.float64 and a.flags.c_contiguous and a.shape == (grid.rows, grid.ny, grid.pitch)
            return ctypes.c_void_p(a.ctypes.data), 0
        return _dev_ptr(a, grid), 1

    def desc(self) -> SolveDesc:
        d = SolveDesc()
        d.grid = self.grid.h
        d.params = params(self.prm)
        d.q0, d.q0_on_device = self._ptr(self.q0, self.grid)
        d.nsteps = self.nsteps
        d.t_end = self.t_end
        d.q_out, d.q_out_on_device = self._ptr(self.q_out, self.grid)
        return d


def padded(grid: Grid, q: np.ndarray) -> np.ndarray:
    """Host state [rows, ny, nx] -> the grid's padded layout [rows, ny, pitch]."""
    out = np.zeros((grid.rows, grid.ny, grid.pitch))
    out[:, :, : grid.nx] = q
    return out


def batch_reserve(ctx: Context, nbytes: int):
    ctx.check(lib().roeam_batch_reserve(ctx.h, int(nbytes)))


def batch_attach(ctx: Context, arena):
    """Run the batch engine over caller-owned device memory: a contiguous torch
    tensor (its storage must outlive the engine; keep a reference)."""
    nbytes = arena.numel() * arena.element_size()
    ctx.check(lib().roeam_batch_attach(ctx.h, ctypes.c_void_p(arena.data_ptr()), int(nbytes)))
    ctx._arena = arena


def batch_configure(ctx: Context, graph_iters: int = 16, persistent: bool = False, policy: int = ADMIT_FIFO,
                    autotune: bool = True, max_resident: int = 0):
    """roeam_batch_configure: iterations per captured graph, persistent batched
    kernels, admission policy (ADMIT_FIFO / ADMIT_SHORTEST), batch tile-shape
    tuning, limit on resident solves (0: none)."""
    ctx.check(lib().roeam_batch_configure(ctx.h, int(graph_iters), int(bool(persistent)), int(policy),
                                          int(bool(autotune)), int(max_resident)))


def batch_info(ctx: Context) -> Dict:
    """roeam_batch_info: graph captures, graph launches, iterations, tunings,
    resident and queued solves, options and the current group tile shape."""
    st = BatchStats()
    ctx.check(lib().roeam_batch_info(ctx.h, ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in BatchStats._fields_}


def batch_descs(solves):
    """The descriptor array of these solves, to submit the same set again
    without rebuilding it (batch_submit(..., descs=))."""
    solves = list(solves)
    return (SolveDesc * len(solves))(*[s.desc() for s in solves])


def batch_submit(ctx: Context, solves, descs=None) -> list:
    solves = list(solves)
    arr = batch_descs(solves) if descs is None else descs
    if len(arr) != len(solves):
        raise ValueError("descs must describe the solves")
    tk = (ctypes.c_uint64 * len(solves))()
    ctx.enter()  # initial states written by the caller's stream are read at admission
    ctx.check(lib().roeam_batch_submit(ctx.h, len(solves), arr, tk))
    for s, t in zip(solves, tk):
        s.ticket = int(t)
    return [int(t) for t in tk]


def batch_run(ctx: Context, iterations: int = -1) -> int:
    pend = ctypes.c_int()
    ctx.enter()
    try:
        ctx.check(lib().roeam_batch_run(ctx.h, int(iterations), ctypes.byref(pend)))
    finally:
        ctx.leave()
    return pend.value


def batch_profile_run(ctx: Context, iterations: int = -1):
    """batch_run with HIP events around every batched stage kernel; returns
    (mean ms of the first to fourth stage launches of a step, number of timed launches)."""
    pend = ctypes.c_int()
    out = (ctypes.c_double * 4)()
    n = ctypes.c_long()
    ctx.enter()
    try:
        ctx.check(lib().roeam_batch_profile_run(ctx.h, int(iterations), ctypes.byref(pend), ctypes.byref(out),
                                                ctypes.byref(n)))
    finally:
        ctx.leave()
    return list(out), n.value


def batch_poll(ctx: Context, ticket: int, leave: bool = True):
    """(done, stats dict or None, status code); a solve that went non-physical
    is done with code ENONPHYS.  leave=False skips the hand-off of a done
    solve's output to torch's current stream: a caller polling many solves
    calls ctx.leave() once afterwards instead (one hand-off covers every
    output the library's stream has written)."""
    done = ctypes.c_int()
    st = StepStats()
    rc = lib().roeam_batch_poll(ctx.h, ctypes.c_uint64(ticket), ctypes.byref(done), ctypes.byref(st))
    if rc not in (OK, ENONPHYS):
        ctx.check(rc)
    if done.value and leave:
        ctx.leave()  # outputs written by the library's stream are read after this
    return bool(done.value), (st.as_dict() if done.value else None), rc


# ---------------------------------------------------------------------------
# 3-D uniform Cartesian grids
# ---------------------------------------------------------------------------

class Grid3:
    """A 3-D uniform Cartesian grid of the library; state tensors are
    [5 + nsc, nz, ny, pitch] (rho, rho u, rho v, rho w, rho E, rho k_m)."""

    def __init__(self, ctx: Context, nx: int, ny: int, nz: int, dx: float, dy: float, dz: float,
                 bc: Sequence[int] = (0,) * 6, bc_state: Optional[np.ndarray] = None):
        self.ctx = ctx
        bca = (ctypes.c_int * 6)(*[int(b) for b in bc])
        st = None
        self._keep = []
        if bc_state is not None:
            sa = np.ascontiguousarray(bc_state, dtype=np.float64).reshape(30)
            self._keep.append(sa)
            st = ctypes.c_void_p(sa.ctypes.data)
        h = ctypes.c_void_p()
        ctx.check(lib().roeam_grid3d_create(ctx.h, int(nx), int(ny), int(nz), float(dx), float(dy), float(dz),
                                            ctypes.byref(bca), st, ctypes.byref(h)))
        self.h = h
        a, b, c, p = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_long()
        lib().roeam_grid3d_layout(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(p))
        self.nx, self.ny, self.nz, self.pitch = a.value, b.value, c.value, p.value
        self.nsc = 0

    @classmethod
    def from_case(cls, ctx: Context, case) -> "Grid3":
        g = cls(ctx, case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, bc=case.bc, bc_state=case.bc_state)
        ns = case.q0.shape[0] - 5
        if ns:
            g.set_scalars(ns, getattr(case, "bc_scalar", None))
        return g

    def set_scalars(self, nscalars: int, bc_scalar: Optional[np.ndarray] = None):
        """Carry nscalars transported scalars (state rows 5..); bc_scalar: [6 sides, nscalars]
        Dirichlet rho k_m."""
        arg = None
        if bc_scalar is not None and nscalars:
            sa = np.ascontiguousarray(np.asarray(bc_scalar, dtype=np.float64)[:, :nscalars]).reshape(-1)
            self._keep.append(sa)
            arg = ctypes.c_void_p(sa.ctypes.data)
        self.ctx.check(lib().roeam_grid3d_set_scalars(self.h, int(nscalars), arg))
        self.nsc = int(nscalars)

    @property
    def rows(self) -> int:
        return 5 + self.nsc

    def empty_state(self):
        import torch
        return torch.zeros((self.rows, self.nz, self.ny, self.pitch), dtype=torch.float64,
                           device=f"cuda:{self.ctx.device}")

    def to_device(self, q: np.ndarray):
        import torch
        t = self.empty_state()
        t[..., : self.nx] = torch.from_numpy(np.ascontiguousarray(q, dtype=np.float64))
        return t

    def from_device(self, t) -> np.ndarray:
        return t[..., : self.nx].detach().cpu().numpy().copy()

    def set_tile_shape(self, shape: int):
        """Shape of the 3-D stage kernel (see SHAPES3; -1: chosen for the grid's size)."""
        self.ctx.check(lib().roeam_grid3d_set_tile_shape(self.h, int(shape)))

    def tile_shape(self, order: int = 2) -> int:
        """The shape the stage kernel runs with for this MUSCL order."""
        out = ctypes.c_int(-1)
        self.ctx.check(lib().roeam_grid3d_tile_shape(self.h, int(order), ctypes.byref(out)))
        return out.value

    def close(self):
        if getattr(self, "h", None):
            lib().roeam_grid3d_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dev_ptr3(t, grid: Grid3) -> ctypes.c_void_p:
    import torch
    assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
    shape = (grid.rows, grid.nz, grid.ny, grid.pitch)
    assert tuple(t.shape) == shape, (tuple(t.shape), shape)
    return ctypes.c_void_p(t.data_ptr())


def residual3(ctx: Context, grid: Grid3, prm: Dict, q, r=None, rate_out=None):
    """R = dQ/dt of the 3-D state tensor q (device, [rows, nz, ny, pitch]); returns r.
    rate_out: optional 1-element float64 device tensor for the max explicit rate."""
    if r is None:
        r = grid.empty_state()
    p = params(prm)
    rp = ctypes.c_void_p(rate_out.data_ptr()) if rate_out is not None else None
    ctx.enter()
    try:
        ctx.check(lib().roeam_residual3d(ctx.h, grid.h, ctypes.byref(p), _dev_ptr3(q, grid), _dev_ptr3(r, grid), rp))
    finally:
        ctx.leave()
    return r


def step3(ctx: Context, grid: Grid3, prm: Dict, q, nsteps: int, t0: float = 0.0, t_end: float = 0.0,
          sync: bool = True) -> Optional[Dict]:
    """Advance the 3-D state q in place; returns the step statistics when sync (else None)."""
    p = params(prm)
    st = StepStats()
    ctx.enter()
    try:
        ctx.check(lib().roeam_step3d(ctx.h, grid.h, ctypes.byref(p), _dev_ptr3(q, grid), int(nsteps), float(t0),
                                     float(t_end), ctypes.byref(st) if sync else None))
    finally:
        ctx.leave()
    return st.as_dict() if sync else None


def last_stats3(ctx: Context, grid: Grid3) -> Dict:
    st = StepStats()
    ctx.check(lib().roeam_last_stats3d(ctx.h, grid.h, ctypes.byref(st)))
    ctx.leave()
    return st.as_dict()
