"""Continuous-batching solve server on top of the batch engine (roeam_batch_*).

Requests (a grid, parameters, a device-resident initial state and a run
length) are admitted by the engine as arena memory frees up; every resident
solve advances one step per scheduler iteration; finished solves are retired
and their output copied out.  The server records each request's submit and
completion wall times, so callers can report latency percentiles beside
throughput.  All solver arithmetic runs in the library's kernels.
"""
from __future__ import annotations

import time
from typing import Dict, List, Optional

import paper_1711_09272_amd as P


class Request:
    def __init__(self, solve: "P.Solve", cells: int, submitted: float, tag=None):
        self.solve = solve
        self.cells = cells
        self.submitted = submitted
        self.finished: Optional[float] = None
        self.stats: Optional[Dict] = None
        self.code: Optional[int] = None
        self.tag = tag

    @property
    def latency(self) -> Optional[float]:
        return None if self.finished is None else self.finished - self.submitted


class Server:
    """One context's batch engine driven as a request loop.

    arena_bytes bounds the device memory held by resident solves (three state
    copies each); requests that do not fit wait in the engine's queue.
    graph_iters: scheduler iterations per captured graph (a finished request
    is noticed after the graph it finished in); policy: admission order of
    queued requests (P.ADMIT_FIFO or P.ADMIT_SHORTEST)."""

    def __init__(self, ctx: "P.Context", arena_bytes: int, graph_iters: int = 8, policy: int = P.ADMIT_FIFO):
        self.ctx = ctx
        P.batch_reserve(ctx, arena_bytes)
        P.batch_configure(ctx, graph_iters=graph_iters, policy=policy)
        self.outstanding: List[Request] = []
        self.done: List[Request] = []

    def submit(self, grid: "P.Grid", prm: Dict, q0, nsteps: int, t_end: float = 0.0, q_out=None,
               tag=None) -> Request:
        if q_out is None:
            q_out = grid.empty_state()
        s = P.Solve(grid, prm, q0, nsteps, t_end, q_out)
        P.batch_submit(self.ctx, [s])
        r = Request(s, grid.nx * grid.ny, time.perf_counter(), tag)
        self.outstanding.append(r)
        return r

    def poll(self) -> List[Request]:
        """Collect requests whose output is written (non-blocking)."""
        fin, keep = [], []
        now = time.perf_counter()
        for r in self.outstanding:
            done, st, code = P.batch_poll(self.ctx, r.solve.ticket)
            if done:
                r.finished, r.stats, r.code = now, st, code
                fin.append(r)
            else:
                keep.append(r)
        self.outstanding = keep
        self.done.extend(fin)
        return fin

    def pump(self, iterations: int = 8) -> List[Request]:
        """Advance the engine by up to `iterations` scheduler iterations, then poll."""
        if self.outstanding:
            P.batch_run(self.ctx, iterations)
        return self.poll()

    def drain(self) -> List[Request]:
        """Run until every submitted request is done."""
        out = []
        while self.outstanding:
            P.batch_run(self.ctx, -1)
            out.extend(self.poll())
        return out
