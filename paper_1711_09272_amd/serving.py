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


class _Lane:
    """One batch engine (its own context, stream and arena) pumped by its own
    host thread; requests reach it through an inbox so that only that thread
    calls into its context."""

    def __init__(self, device: int, arena_bytes: int, graph_iters: int, max_resident: int):
        import collections
        import threading
        self.server = Server(P.Context(device), arena_bytes, graph_iters=graph_iters)
        if max_resident:
            P.batch_configure(self.server.ctx, graph_iters=graph_iters, max_resident=max_resident)
        self.graph_iters = graph_iters
        self.inbox = collections.deque()
        self.done: List[Request] = []
        self.error: Optional[BaseException] = None
        self._stop = False
        self._thread = threading.Thread(target=self._run, daemon=True)
        self._thread.start()

    def _run(self):
        try:
            while not self._stop or self.inbox or self.server.outstanding:
                while self.inbox:
                    req, grid, prm, q0, nsteps, t_end, q_out = self.inbox.popleft()
                    if q_out is None:
                        q_out = grid.empty_state()
                    req.solve = P.Solve(grid, prm, q0, nsteps, t_end, q_out)
                    P.batch_submit(self.server.ctx, [req.solve])
                    self.server.outstanding.append(req)
                if self.server.outstanding:
                    self.done.extend(self.server.pump(self.graph_iters))
                else:
                    time.sleep(0.0002)
        except BaseException as e:  # surfaced by the caller's next call
            self.error = e

    def stop(self):
        self._stop = True
        self._thread.join()


class SplitServer:
    """Requests served on two batch engines of one GPU, each on its own stream
    and pumped by its own host thread: solves of fewer than `split_cells`
    cells run batched together in the small lane; larger ones queue for the
    large lane, which holds at most `large_resident` of them at a time (one:
    the large solves run one after another, nearly alone).  The lanes' graphs
    run side by side on the device, so a small solve is no longer paced by the
    step time of the largest grid resident with it (in one engine every
    resident solve takes one step per iteration), and a large solve shares the
    device only with small ones.  Results are bitwise those of the solves run
    alone (same kernels)."""

    def __init__(self, device: int, arena_bytes: int, split_cells: int = 512 * 512, large_resident: int = 1,
                 graph_iters: int = 8):
        self.split_cells = split_cells
        self.small = _Lane(device, arena_bytes // 2, graph_iters, 0)
        self.large = _Lane(device, arena_bytes // 2, graph_iters, large_resident)
        self.requests: List[Request] = []

    def submit(self, grid: "P.Grid", prm: Dict, q0, nsteps: int, t_end: float = 0.0, q_out=None,
               tag=None) -> Request:
        for lane in (self.small, self.large):
            if lane.error:
                raise lane.error
        lane = self.small if grid.nx * grid.ny < self.split_cells else self.large
        r = Request(None, grid.nx * grid.ny, time.perf_counter(), tag)
        lane.inbox.append((r, grid, prm, q0, nsteps, t_end, q_out))
        self.requests.append(r)
        return r

    @property
    def outstanding(self) -> int:
        for lane in (self.small, self.large):
            if lane.error:
                raise lane.error
        return len(self.requests) - len(self.small.done) - len(self.large.done)

    def drain(self, poll_s: float = 0.0005):
        while self.outstanding:
            time.sleep(poll_s)

    def close(self):
        self.small.stop()
        self.large.stop()
        for lane in (self.small, self.large):
            if lane.error:
                raise lane.error
