#!/usr/bin/env python
"""Throughput of the Roe-AM step on one MI355X: Gcell-updates/s per RK stage.

Default workload (the low-Mach vortex configuration): two 256 x 256 periodic
grids, free-stream Mach 0.01 and 0.001, FP64, MUSCL-minmod + SSP-RK3, full
Roe-AM (detector on, eps1 = 1, eps2 = 0.05), CFL 0.4 with the c / sqrt(theta)
time-step rule, seeded +-1e-6 pressure checkerboard.  Both grids advance
together through the batch engine (one batched stage kernel per RK stage, each
grid with its own dt); one bench step is one SSP-RK3 step of both grids.
Inputs are resident in HBM before the timed region.  `--workload vortexN`
runs one N x N grid (M = 0.01) through roeam_step instead.

Prints one JSON line.  Extra legs: the roofline of the stage kernel (HIP events
around each stage launch of the same grid launched alone), and the CPU oracle
on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# Algorithmic HBM bytes per cell for one SSP-RK3 step: stage 1 reads Q and
# writes Q1 (64 B); stages 2 and 3 read the stage input and Q^n and write the
# result (96 B each).  Per stage launch on average: 256/3 B per cell.
BYTES_PER_CELL_STAGE = {1: 64.0, 2: 96.0, 3: 96.0}


# 3-D: five rows; stage 1 reads Q and writes Q1 (80 B), stages 2 and 3 read the
# stage input and Q^n and write the result (120 B each).
BYTES_PER_CELL_STAGE_3D = {1: 80.0, 2: 120.0, 3: 120.0}


# The device code of the stage kernels: counter summaries taken on other
# sources are stale.  (Host-side scheduling files are not part of the hash.)
KERNEL_SOURCES = ("roeam_kernels.hip", "roeam_stage2d.hpp", "roeam_device.hpp", "roeam_stage.hpp")
KERNEL_SOURCES_3D = ("roeam_kernels3d.hip", "roeam_stage3d.hpp", "roeam_device3d.hpp", "roeam_device.hpp",
                     "roeam_stage.hpp")


def is_3d(workload: str) -> bool:
    return workload.startswith("vortex3d")


def kernel_source_hash(sources=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1711_09272_amd", "csrc")
    for name in sources:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_summary(workload: str, precision: int, kind: str, key: str):
    """One figure of a committed rocprofv3 counter summary (profiles/), or None
    when it is missing or was taken on a different kernel source."""
    tag = workload + ("_fp32coef" if precision else "")
    path = os.path.join(ROOT, "profiles", f"stage_kernel_{tag}_{kind}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        parts = line.split()
        if len(parts) >= 2 and not line.startswith("#"):
            vals[parts[0]] = parts[1]
    if vals.get("kernel_source_hash") != kernel_source_hash(KERNEL_SOURCES_3D if is_3d(workload) else KERNEL_SOURCES):
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def measured_traffic(workload: str, precision: int):
    """HBM bytes per stage launch (FETCH_SIZE and WRITE_SIZE passes, scaled)."""
    return counter_summary(workload, precision, "traffic", "hbm_bytes_per_launch")


def measured_valu(workload: str, precision: int):
    """VALU lane-instructions per cell-stage (SQ_INSTS_VALU x 64 / cells)."""
    return counter_summary(workload, precision, "valu", "valu_lane_instr_per_cell_stage")


# VALU issue ceiling: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz (one
# wave64 VALU instruction per SIMD every 4 clocks; an FP64 FMA is one such
# instruction, which is where 78.6 TFLOP/s FP64 comes from).
PEAK_VALU_LANE_INSTR = 256 * 4 * 16 * 2.4e9


def make_cases(workload: str, precision: int, order=None, eps1=None, time_scheme=None):
    """The grids of a workload (list) and whether they run as one batch
    (order / eps1: overrides of the workload's MUSCL order and eps1)."""
    import workloads
    if workload == "vortex256pair":
        cases = [workloads.vortex(256, 0.01), workloads.vortex(256, 0.001)]
        batched = True
    elif workload.startswith("vortex"):
        cases = [workloads.vortex(int(workload[len("vortex"):]), 0.01)]
        batched = False
    else:
        raise SystemExit(f"unknown workload {workload}")
    for c in cases:
        c.params["precision"] = precision
        if order is not None:
            c.params["order"] = order
        if eps1 is not None:
            c.params["eps1"] = eps1
        if time_scheme is not None:
            c.params["time_scheme"] = time_scheme
    return cases, batched


def cpu_baseline(cases, sample_steps: int):
    """The oracle as it stands on this host: all its OpenMP threads (the reported
    value; its row loops give the same bits for any thread count), and one
    thread on a shorter sample."""
    import oracle

    def timed(steps):
        t0 = time.perf_counter()
        updates = 0
        for case in cases:
            _, st = oracle.run(case, nsteps=steps)
            updates += case.nx * case.ny * 3 * st["steps"]
        return updates, time.perf_counter() - t0

    names = " + ".join(f"{c.nx}x{c.ny} M={c.params['mach_ref']:g}" for c in cases)
    threads = oracle.max_threads()
    single_steps = max(min(sample_steps, 50), 1)
    oracle.set_threads(1)
    u1, dt1 = timed(single_steps)
    oracle.set_threads(threads)
    un, dtn = timed(sample_steps)
    return {
        "value": un / dtn / 1e9,
        "unit": "Gcell-updates/s per RK stage",
        "cores": threads,
        "kind": "oracle",
        "sample": f"first {sample_steps} SSP-RK3 steps of each grid of the same workload ({names}; "
                  f"{un} cell-stage updates, {dtn:.1f} s, {threads} OpenMP threads over rows)",
        "single_thread": {"value": u1 / dt1 / 1e9, "cores": 1,
                          "sample": f"first {single_steps} steps of each grid, {u1} cell-stage updates, {dt1:.1f} s"},
    }


def spin_up(chunk, seconds: float) -> int:
    """Bring the GPU to its sustained clocks before anything is timed: run
    `chunk` (a piece of the workload's own GPU work that synchronises) until
    `seconds` of wall time have passed; returns the number of chunks.  On a
    fresh box the first seconds of light, bursty load run at low clocks (the
    2 x 256^2 pair measured 3.4x slower in the first bench processes of a new
    box), and W warm-up steps of a fast kernel are only milliseconds of work."""
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        chunk()
        n += 1
    return n


def spin_up_generic(seconds: float) -> int:
    """The same with FP64 matrix products (modes whose own work is real-time driven)."""
    import torch
    x = torch.rand(2048, 2048, dtype=torch.float64, device="cuda")

    def chunk():
        for _ in range(4):
            torch.mm(x, x)
        torch.cuda.synchronize()
    return spin_up(chunk, seconds)


def timed_batch(ctx, grids, cases, steps, warmup, stream, spin_s=0.0):
    """Advance every grid `steps` steps together through the batch engine;
    returns GPU ms between events around submission and completion."""
    import torch
    import paper_1711_09272_amd as P
    # tune the tile shape on the first grid (a zero-step run); the batch uses it
    P.step(ctx, grids[0], cases[0].params, grids[0].to_device(cases[0].q0), 0)
    q0 = [g.to_device(c.q0) for g, c in zip(grids, cases)]
    qout = [g.empty_state() for g in grids]
    P.batch_reserve(ctx, sum(g.footprint() for g in grids) + (1 << 20))

    def run(n):
        solves = [P.Solve(g, c.params, q, n, 0.0, o) for g, c, q, o in zip(grids, cases, q0, qout)]
        P.batch_submit(ctx, solves)
        P.batch_run(ctx, -1)
        return solves

    spin_up(lambda: (run(100), torch.cuda.synchronize()), spin_s)
    run(warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    solves = run(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for s in solves:
        done, st, rc = P.batch_poll(ctx, s.ticket)
        if not done or rc != P.OK or st["steps"] != steps:
            raise SystemExit(f"bench batch run failed: {done} {st} {rc}")
    return ev0.elapsed_time(ev1), wall


def profile_batch(ctx, grids, cases, steps):
    """The same batch again for `steps` steps with HIP events around every
    batched stage launch (on the library's stream); (stage ms, launches)."""
    import paper_1711_09272_amd as P
    q0 = [g.to_device(c.q0) for g, c in zip(grids, cases)]
    solves = [P.Solve(g, c.params, q, steps, 0.0, g.empty_state()) for g, c, q in zip(grids, cases, q0)]
    P.batch_submit(ctx, solves)
    stage_ms, launches = P.batch_profile_run(ctx, -1)
    for s in solves:
        done, st, rc = P.batch_poll(ctx, s.ticket)
        if not done or rc != P.OK or st["steps"] != steps:
            raise SystemExit(f"bench batch profile run failed: {done} {st} {rc}")
    return stage_ms, launches


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q)) if xs else None


def one_at_a_time(ctx, items, precision):
    """Run each (grid, params, q0_tensor, steps) alone through roeam_step in
    order; returns per-item GPU-serial completion times (s from start) and total.
    Tile shapes are tuned and the step graphs captured beforehand (a run of up
    to 50 steps of each item on its own working buffer, which the timed run
    reuses), so the timed runs only replay graphs."""
    import torch
    import paper_1711_09272_amd as P
    bufs = []
    for g, prm, q0, n in items:
        p = dict(prm)
        p["precision"] = precision
        b = q0.clone()
        P.step(ctx, g, p, b, min(n, 50), sync=True)
        bufs.append(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = []
    for (g, prm, q0, n), b in zip(items, bufs):
        p = dict(prm)
        p["precision"] = precision
        b.copy_(q0)
        P.step(ctx, g, p, b, n, sync=True)
        done.append(time.perf_counter() - t0)
    return done, time.perf_counter() - t0


def batch_cases(n_grids: int, prec: int):
    """The fourth configuration's grids: 256 bump-family periodic grids, sides
    log-uniform 32..512 (seeded), MUSCL + SSP-RK3, 200 steps each."""
    import workloads
    return workloads.batch_family(n_grids, nsteps=BATCH_STEPS, precision=prec)


BATCH_STEPS = 200
BATCH_GRAPH_ITERS = 20  # 200 steps = 10 graphs


class BatchRunner:
    """The fourth configuration on the batch engine: all grids submitted at
    once and advanced together until every one is done; one `run` is one
    bench step (the whole batch, 200 SSP-RK3 steps of each grid)."""

    def __init__(self, ctx, cases, persistent=False, reserve_extra=64 << 20):
        import paper_1711_09272_amd as P
        self.P, self.ctx, self.cases = P, ctx, cases
        self.grids = [P.Grid.from_case(ctx, c) for c in cases]
        self.q0 = [g.to_device(c.q0) for g, c in zip(self.grids, cases)]
        self.out = [g.empty_state() for g in self.grids]
        self.cells = sum(c.nx * c.ny for c in cases)
        P.batch_reserve(ctx, sum(g.footprint() for g in self.grids) + reserve_extra)
        P.batch_configure(ctx, graph_iters=BATCH_GRAPH_ITERS, persistent=persistent)
        self._sets = {}  # run length -> (solves, their descriptor array), built once

    def run(self, nsteps=BATCH_STEPS):
        """Submit every grid, drive the engine until all are done; returns the
        latency of each solve (s, submission to the poll that saw it done).
        The Python solve objects and their descriptor array are built once per
        run length and submitted again on each call (the engine copies each
        initial state into its arena at admission)."""
        P = self.P
        if nsteps not in self._sets:
            solves = [P.Solve(g, c.params, q, nsteps, 0.0, o)
                      for g, c, q, o in zip(self.grids, self.cases, self.q0, self.out)]
            self._sets[nsteps] = (solves, P.batch_descs(solves))
        solves, descs = self._sets[nsteps]
        t0 = time.perf_counter()
        P.batch_submit(self.ctx, solves, descs=descs)
        fin = {}
        while len(fin) < len(solves):
            P.batch_run(self.ctx, BATCH_GRAPH_ITERS)
            now = time.perf_counter()
            n0 = len(fin)
            for s in solves:
                if s.ticket not in fin:
                    done, st, rc = P.batch_poll(self.ctx, s.ticket, leave=False)
                    if done:
                        if rc != P.OK or st["steps"] != nsteps:
                            raise SystemExit(f"batched solve failed: {st} {rc}")
                        fin[s.ticket] = now - t0
            if len(fin) > n0:
                self.ctx.leave()  # the finished solves' outputs, handed to torch's stream once
        return [fin[s.ticket] for s in solves]

    def profile(self, nsteps=BATCH_STEPS):
        """The same batch once more with HIP events around every batched stage
        launch (direct launches, no graph): (mean stage ms, launches)."""
        P = self.P
        solves = [P.Solve(g, c.params, q, nsteps, 0.0, o)
                  for g, c, q, o in zip(self.grids, self.cases, self.q0, self.out)]
        P.batch_submit(self.ctx, solves)
        stage_ms, launches = P.batch_profile_run(self.ctx, -1)
        for s in solves:
            done, st, rc = P.batch_poll(self.ctx, s.ticket)
            if not done or rc != P.OK or st["steps"] != nsteps:
                raise SystemExit(f"batched profile run failed: {done} {st} {rc}")
        return stage_ms, launches


def timed_repeats(fn, k, stream):
    """GPU seconds (HIP events on torch's stream, which waits for the library's
    stream before the end event) and wall seconds of k calls of fn; also the
    list of fn's results."""
    import torch
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    res = [fn() for _ in range(k)]
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / 1e3, time.perf_counter() - t0, res


def single_grid_point(ctx, n, steps, precision, stream):
    """One n x n vortex grid through roeam_step (autotuned shape, graph
    replay): Gcell-stage/s and the HBM fraction of the stage kernel."""
    import torch
    import paper_1711_09272_amd as P
    import workloads
    case = workloads.vortex(n, 0.01)
    case.params["precision"] = precision
    g = P.Grid.from_case(ctx, case)
    q = g.to_device(case.q0)
    P.step(ctx, g, case.params, q, 20, sync=True)  # tunes the shape, captures the graph
    gpu_s, wall, _ = timed_repeats(lambda: P.step(ctx, g, case.params, q, steps, sync=False), 1, stream)
    st = P.last_stats(ctx, g)
    if st["nonphys"] or st["steps"] != steps:
        raise SystemExit(f"single-grid run failed: {st}")
    cells = n * n
    launch_ms = gpu_s * 1e3 / (3 * steps)
    bytes_per_launch = cells * sum(BYTES_PER_CELL_STAGE.values()) / 3.0
    achieved = bytes_per_launch / (launch_ms / 1e3) / 1e9
    shape = g.tile_shape(case.params)
    return {"workload": f"low-Mach vortex {n}x{n} periodic, M=0.01, MUSCL + SSP-RK3, Roe-AM (detector, eps1=1)",
            "dtype": "f64" if precision == 0 else "f32-flux/f64-state", "steps": steps,
            "value": round(cells * 3 * steps / gpu_s / 1e9, 4), "unit": "Gcell-updates/s",
            "ms_per_step": round(gpu_s * 1e3 / steps, 5), "tile_shape": P.SHAPES[shape] if shape >= 0 else None,
            "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": round(achieved / PEAK_HBM_GBS, 5), "launch_ms": round(launch_ms, 6),
                         "algorithmic_bytes_per_launch": bytes_per_launch}}


def bench_batch(args):
    """Fourth configuration (the default line): 256 seeded grids of sides
    log-uniform 32..512, 200 SSP-RK3 steps each, FP32 flux coefficients with
    FP64 state, all submitted at once and advanced together through the batch
    engine (graph-replayed batched stage kernels).  A bench step is the whole
    batch; --steps and --warmup count whole batches."""
    import torch
    import paper_1711_09272_amd as P
    prec = 1 if args.precision is None else args.precision
    cases = batch_cases(args.batch_grids, prec)
    ctx = P.Context(0)
    stream = torch.cuda.current_stream()
    runner = BatchRunner(ctx, cases, persistent=args.batch_persistent)
    cells = runner.cells
    updates_per_step = cells * 3 * BATCH_STEPS
    bytes_per_launch = cells * sum(BYTES_PER_CELL_STAGE.values()) / 3.0
    if args.counter_run:
        stage_ms, launches = runner.profile(args.profile_steps)
        src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")  # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"counter_run": "batch256", "cells": cells, "profile_steps": args.profile_steps,
                          "copy_bytes": src.numel() * 8, "info": P.batch_info(ctx)}), flush=True)
        return
    spin_up(lambda: runner.run(20), args.spin_up_s)
    for _ in range(max(args.warmup, 1)):  # the first forms the group: tile-shape tuning, graph capture
        runner.run()
    info0 = P.batch_info(ctx)
    gpu_s, wall, lats = timed_repeats(runner.run, args.steps, stream)
    info = P.batch_info(ctx)
    lat = [x for rep in lats for x in rep]
    launches_per_step = 3 * BATCH_STEPS
    launch_ms = gpu_s * 1e3 / (args.steps * launches_per_step)
    achieved = bytes_per_launch / (launch_ms / 1e3) / 1e9
    stage_ms, plaunches = runner.profile()
    tag = "batch256"
    traffic = measured_traffic(tag, prec)
    valu = measured_valu(tag, prec)
    alu = None
    if valu is not None:
        lane_rate = valu * cells / (launch_ms / 1e3)
        alu = {"bound": "alu", "achieved": round(lane_rate / 1e12, 3), "peak": round(PEAK_VALU_LANE_INSTR / 1e12, 3),
               "unit": "T VALU lane-instr/s", "frac": round(lane_rate / PEAK_VALU_LANE_INSTR, 4),
               "valu_lane_instr_per_cell_stage": valu}
    shape = info["shape"]
    kform = "k_stage_batch_p" if args.batch_persistent else "k_stage_batch"
    out = {
        "metric": "Gcell-updates/s per RK stage",
        "value": round(updates_per_step * args.steps / gpu_s / 1e9, 4),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(gpu_s * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32-flux/f64-state",
        "data": "synthetic",
        "config": {"workload": f"{len(cases)} bump-family periodic grids, sides log-uniform 32..512 (seeded), "
                               f"{BATCH_STEPS} SSP-RK3 steps each, MUSCL-minmod, Roe-AM (detector, eps1=1), "
                               "submitted together, continuous-batching engine; one bench step = the whole batch",
                   "grids": len(cases), "cells": cells, "rk_steps_per_grid": BATCH_STEPS,
                   "cell_stage_updates_per_step": updates_per_step,
                   "tile_shape": P.SHAPES[shape] if shape >= 0 else None,
                   "kernel_form": "persistent" if args.batch_persistent else "one workgroup per tile",
                   "graph_iters": BATCH_GRAPH_ITERS, "graph_captures_in_timed_region": info["captures"] - info0["captures"],
                   "wall_s": round(wall, 4)},
        "latency_s": {"p50": percentile(lat, 50), "p99": percentile(lat, 99), "max": max(lat),
                      "what": "per solve, submission to completion, every solve of every timed batch"},
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 2),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 5),
            "traffic": traffic,
            "traffic_frac": round(traffic / (launch_ms / 1e3) / 1e9 / PEAK_HBM_GBS, 5) if traffic else None,
            "alu": alu,
            "kernel": "%s<order 2, FP%s, uniform, %s>" % (kform, "64" if prec == 0 else "32-coef",
                                                         P.SHAPES[shape] if shape >= 0 else "?"),
            "kernel_grid": f"{len(cases)} grids, {cells} cells",
            "launch_ms": round(launch_ms, 6),
            "timed_region_launches": args.steps * launches_per_step,
            "event_bracketed_stage_ms": [round(x, 5) for x in stage_ms[:3]],
            "event_bracketed_launches": plaunches,
            "algorithmic_bytes_per_launch": bytes_per_launch,
        },
    }
    if not args.no_extra_legs:
        # the same batch in FP64
        cases64 = batch_cases(args.batch_grids, 0)
        r64 = BatchRunner(ctx, cases64, persistent=args.batch_persistent)
        r64.run()
        k64 = max(1, args.steps // 4)
        g64, _, lats64 = timed_repeats(r64.run, k64, stream)
        lat64 = [x for rep in lats64 for x in rep]
        out["fp64"] = {"value": round(updates_per_step * k64 / g64 / 1e9, 4), "ms_per_step": round(g64 * 1e3 / k64, 4),
                       "repeats": k64, "latency_p50_s": percentile(lat64, 50), "latency_p99_s": percentile(lat64, 99),
                       "hbm_frac": round(bytes_per_launch / (g64 / (k64 * launches_per_step)) / 1e9 / PEAK_HBM_GBS, 5)}
        del r64
        # one grid at a time through roeam_step, shapes tuned and graphs captured beforehand
        items = [(g, c.params, q, BATCH_STEPS) for g, c, q in zip(runner.grids, cases, runner.q0)]
        legs = {}
        for name, pr in (("fp64", 0), ("same_precision", prec)):
            done, total = one_at_a_time(ctx, items, pr)
            legs[name] = {"value": round(updates_per_step / total / 1e9, 4), "makespan_s": round(total, 4),
                          "p50_s": percentile(done, 50), "p99_s": percentile(done, 99)}
        out["one_at_a_time"] = legs
        # the single-grid FP64 path at 2048^2
        out["single_grid_fp64_2048"] = single_grid_point(ctx, 2048, args.single_steps, 0, stream)
    if not args.no_cpu_baseline:
        # the oracle on a bounded sample: the first 16 grids, all their steps, FP64
        import oracle
        sample = cases[:16]
        t0 = time.perf_counter()
        upd = 0
        for c in sample:
            prm = dict(c.params)
            prm["precision"] = 0
            _, st = oracle.run(c, params=prm, nsteps=BATCH_STEPS)
            upd += c.nx * c.ny * 3 * st["steps"]
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": upd / dt / 1e9, "unit": "Gcell-updates/s per RK stage",
                               "cores": oracle.max_threads(), "kind": "oracle",
                               "sample": f"the first {len(sample)} of the {len(cases)} grids, {BATCH_STEPS} steps each, "
                                         f"FP64 ({upd} cell-stage updates, {dt:.1f} s, "
                                         f"{oracle.max_threads()} OpenMP threads over rows)"}
    print(json.dumps(out), flush=True)


def bench_to_t_end(args):
    """The first and third configurations, each run to its end time through
    roeam_step: Sod 400 x 4 (first order, forward Euler, to t = 0.2) and the
    Mach-20 odd-even channel 800 x 80 (MUSCL, SSP-RK3, node grid, to t = 30).
    The oracle runs the same case in full for the CPU baseline."""
    import torch
    import paper_1711_09272_amd as P
    import workloads
    case = workloads.sod() if args.workload == "sod" else workloads.odd_even()
    if args.precision:
        case.params["precision"] = args.precision
    stages = {0: 1, 1: 3, 2: 4}[case.params["time_scheme"]]
    ctx = P.Context(0)
    g = P.Grid.from_case(ctx, case)
    stream = torch.cuda.current_stream()
    spin_up(lambda: P.step(ctx, g, case.params, g.to_device(case.q0), 200, 0.0, case.t_end, sync=True),
            args.spin_up_s)
    times = []
    for rep in range(2):  # the first run tunes the tile shape and captures graphs
        q = g.to_device(case.q0)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        P.step(ctx, g, case.params, q, case.nsteps, 0.0, case.t_end, sync=False)
        ev1.record(stream)
        st = P.last_stats(ctx, g)
        torch.cuda.synchronize()
        times.append(ev0.elapsed_time(ev1) / 1e3)
        if st["nonphys"] or st["t"] != case.t_end:
            raise SystemExit(f"run failed: {st}")
    gpu_s = times[-1]
    updates = case.nx * case.ny * stages * st["steps"]
    shape = g.tile_shape(case.params)
    out = {
        "metric": "Gcell-updates/s per RK stage",
        "value": round(updates / gpu_s / 1e9, 4),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": st["steps"],
        "ms_per_step": round(gpu_s * 1e3 / st["steps"], 5),
        "higher_is_better": True,
        "dtype": "f64" if not args.precision else "f32-flux/f64-state",
        "data": "synthetic",
        "config": {"workload": ("Sod shock tube 400x4, first order, forward Euler, CFL 0.4, to t = 0.2"
                                if args.workload == "sod" else
                                "Mach-20 odd-even channel 800x80 (node grid, centreline +-1e-6), MUSCL + "
                                "SSP-RK3, CFL 0.4, to t = 30"),
                   "cells": case.nx * case.ny, "stages_per_step": stages, "t_end": case.t_end,
                   "tile_shape": P.SHAPES[shape] if shape >= 0 else None, "run_s": round(gpu_s, 5)},
    }
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        _, st_or = oracle.run(case)
        dt = time.perf_counter() - t0
        upd = case.nx * case.ny * stages * st_or["steps"]
        out["cpu_baseline"] = {"value": upd / dt / 1e9, "unit": "Gcell-updates/s per RK stage",
                               "cores": oracle.max_threads(), "kind": "oracle",
                               "sample": f"the whole run ({st_or['steps']} steps, {upd} cell-stage updates, {dt:.1f} s)"}
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Fifth configuration: Poisson arrivals (rates swept) of solves with grid
    sides log-uniform 64..2048 and 50..2000 steps, bump-family states; served
    with continuous batching vs one at a time through roeam_step.  Initial
    states are built on the device before each trace starts; the
    one-at-a-time leg has every grid size's tile shape tuned and step graph
    captured beforehand, so neither leg pays set-up inside a latency."""
    import torch
    import paper_1711_09272_amd as P
    import workloads
    from paper_1711_09272_amd.serving import Server, SplitServer
    prec = 0 if args.precision is None else args.precision
    ctx = P.Context(0)
    grid_cache, buf_cache = {}, {}

    def grid(n):
        if n not in grid_cache:
            grid_cache[n] = P.Grid(ctx, n, n, dx=1.0 / n, dy=1.0 / n, bc=(0, 0, 0, 0))
        return grid_cache[n]

    spin_up_generic(args.spin_up_s)
    results = []
    work_total = 0.0
    for rate in [float(r) for r in args.rates.split(",")]:
        trace = workloads.serving_trace(rate, args.duration)
        states = [workloads.bump_state_device(tr["n"], tr["spec"], grid(tr["n"]).pitch) for tr in trace]
        prms = [workloads.bump_params(tr["spec"]["mach"], precision=prec) for tr in trace]
        # one-at-a-time set-up, outside any latency: tune each size's tile shape
        # and capture its step graph on a working buffer of that size
        for tr, q0, prm in zip(trace, states, prms):
            n = tr["n"]
            if n not in buf_cache:
                buf_cache[n] = q0.clone()
                P.step(ctx, grid(n), prm, buf_cache[n], 50, sync=True)
        torch.cuda.synchronize()
        legs = {}
        for leg in ("served_split", "served", "one_at_a_time"):
            t0 = time.perf_counter()
            lat, done_at = [], []
            if leg == "served_split":
                srv = SplitServer(0, args.arena_gb << 30, split_cells=args.split_cells,
                                  graph_iters=args.serve_graph_iters)
                k = 0
                reqs = []
                while k < len(trace) or srv.outstanding:
                    now = time.perf_counter() - t0
                    while k < len(trace) and trace[k]["arrival_s"] <= now:
                        r = srv.submit(grid(trace[k]["n"]), prms[k], states[k], trace[k]["steps"], tag=k)
                        r.arrival = t0 + trace[k]["arrival_s"]
                        reqs.append(r)
                        k += 1
                    time.sleep(0.0005)
                srv.close()
                lat = [r.finished - r.arrival for r in reqs]
                done_at = [r.finished for r in reqs]
                bad = [r for r in reqs if r.code != P.OK or r.stats["steps"] != r.solve.nsteps]
                if bad:
                    raise SystemExit(f"served request failed: {bad[0].stats} {bad[0].code}")
                for r in reqs:
                    r.solve.q_out = None
                del srv
            elif leg == "served":
                server = Server(ctx, args.arena_gb << 30, graph_iters=args.serve_graph_iters, policy=args.serve_policy)
                k = 0
                reqs = []
                while k < len(trace) or server.outstanding:
                    now = time.perf_counter() - t0
                    while k < len(trace) and trace[k]["arrival_s"] <= now:
                        r = server.submit(grid(trace[k]["n"]), prms[k], states[k], trace[k]["steps"], tag=k)
                        r.arrival = t0 + trace[k]["arrival_s"]
                        reqs.append(r)
                        k += 1
                    if server.outstanding:
                        for r in server.pump(args.serve_graph_iters):
                            r.solve.q_out = None  # release device memory
                    else:
                        time.sleep(0.0005)
                lat = [r.finished - r.arrival for r in reqs]
                done_at = [r.finished for r in reqs]
                bad = [r for r in reqs if r.code != P.OK or r.stats["steps"] != r.solve.nsteps]
                if bad:
                    raise SystemExit(f"served request failed: {bad[0].stats} {bad[0].code}")
                del server
            else:
                for tr, q0, prm in zip(trace, states, prms):
                    wait = t0 + tr["arrival_s"] - time.perf_counter()
                    if wait > 0:
                        time.sleep(wait)
                    b = buf_cache[tr["n"]]
                    b.copy_(q0)
                    st = P.step(ctx, grid(tr["n"]), prm, b, tr["steps"], sync=True)
                    if st["nonphys"] or st["steps"] != tr["steps"]:
                        raise SystemExit(f"one-at-a-time request failed: {st}")
                    now = time.perf_counter()
                    lat.append(now - (t0 + tr["arrival_s"]))
                    done_at.append(now)
            updates = sum(tr["n"] * tr["n"] * 3 * tr["steps"] for tr in trace)
            span = max(done_at) - (t0 + trace[0]["arrival_s"])
            legs[leg] = {"gcell_updates_per_s": round(updates / span / 1e9, 4), "p50_s": percentile(lat, 50),
                         "p99_s": percentile(lat, 99), "mean_s": sum(lat) / len(lat), "span_s": round(span, 3)}
        work = sum(tr["n"] * tr["n"] * 3 * tr["steps"] for tr in trace)
        work_total += work
        results.append({"rate_per_s": rate, "requests": len(trace), "duration_s": args.duration,
                        "cell_stage_updates": work, "served_two_lanes": legs["served_split"],
                        "served_one_engine": legs["served"], "one_at_a_time": legs["one_at_a_time"]})
        print(json.dumps({"serve_rate": rate, **results[-1]}), file=sys.stderr, flush=True)
        del states
        torch.cuda.synchronize()
    out = {"metric": "served p50/p99 latency and Gcell-updates/s", "n_gpus": 1,
           "dtype": "f64" if prec == 0 else "f32-flux/f64-state", "data": "synthetic",
           "config": {"workload": "Poisson requests, sides log-uniform 64..2048, steps log-uniform 50..2000, "
                                  "bump-family states, SSP-RK3 + MUSCL; continuous batching (two lanes: solves "
                                  f"below {args.split_cells} cells batched together, larger ones one at a time beside "
                                  "them; and one engine for all) vs one request at a time",
                      "arena_gb": args.arena_gb, "graph_iters": args.serve_graph_iters,
                      "admission": "shortest-first" if args.serve_policy == P.ADMIT_SHORTEST else "fifo"},
           "rates": results}
    if not args.no_cpu_baseline:
        # the oracle's per-cell-stage cost on a sample of the same state family
        # (the first 4 grids of the batched configuration, 200 steps, FP64),
        # extrapolated to each trace's work: an extrapolation, not a run
        import oracle
        sample = batch_cases(4, 0)
        t0 = time.perf_counter()
        upd = 0
        for c in sample:
            _, st = oracle.run(c, nsteps=BATCH_STEPS)
            upd += c.nx * c.ny * 3 * st["steps"]
        dt = time.perf_counter() - t0
        rate_or = upd / dt
        out["cpu_baseline"] = {"value": rate_or / 1e9, "unit": "Gcell-updates/s per RK stage",
                               "cores": oracle.max_threads(), "kind": "oracle",
                               "sample": f"4 grids of the bump family (sides {[c.nx for c in sample]}), "
                                         f"{BATCH_STEPS} steps each, FP64 ({upd} cell-stage updates, {dt:.1f} s)",
                               "extrapolated_trace_s": {str(r["rate_per_s"]): round(r["cell_stage_updates"] / rate_or, 1)
                                                        for r in results}}
    print(json.dumps(out), flush=True)


def parse_3d(workload: str):
    """vortex3dNxNZ -> (N, NZ)."""
    dims = workload[len("vortex3d"):].split("x")
    if len(dims) != 2:
        raise SystemExit(f"unknown workload {workload} (3-D form: vortex3dNxNZ)")
    return int(dims[0]), int(dims[1])


def cpu_baseline_3d(case, sample_steps: int):
    import oracle
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    _, st = oracle.run3(case, nsteps=sample_steps)
    dt = time.perf_counter() - t0
    updates = case.cells * 3 * st["steps"]
    return {
        "value": updates / dt / 1e9,
        "unit": "Gcell-updates/s per RK stage",
        "cores": threads,
        "kind": "oracle",
        "sample": f"first {sample_steps} SSP-RK3 steps of the same {case.nx}x{case.ny}x{case.nz} grid "
                  f"({updates} cell-stage updates, {dt:.1f} s, {threads} OpenMP threads over z-planes)",
    }


def bench_3d(args):
    """One 3-D grid: the vortex extruded along a periodic z with a seeded w and
    +-1e-6 checkerboard (all three face directions and the nine-face detector
    active), through roeam_step3d."""
    import torch
    import paper_1711_09272_amd as P
    import workloads
    n, nz = parse_3d(args.workload)
    case = workloads.vortex3(n, nz, 0.01, time_scheme=1, precision=args.precision)
    cells = case.cells
    ctx = P.Context(0)
    grid = P.Grid3.from_case(ctx, case)
    grid.set_tile_shape(args.tile_shape)  # -1: the shape chosen for the grid's size
    shape = grid.tile_shape(case.params["order"])
    q = grid.to_device(case.q0)
    prm = case.params
    stream = torch.cuda.current_stream()
    if args.counter_run:
        P.step3(ctx, grid, prm, q, args.profile_steps, sync=True)
        src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")  # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"counter_run": args.workload, "cells": cells, "profile_steps": args.profile_steps,
                          "copy_bytes": src.numel() * 8, "tile_shape": P.SHAPES3[shape]}), flush=True)
        return
    q_spin = grid.to_device(case.q0)
    spin_up(lambda: P.step3(ctx, grid, prm, q_spin, 4, sync=True), args.spin_up_s)
    del q_spin
    P.step3(ctx, grid, prm, q, args.warmup, sync=True)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    P.step3(ctx, grid, prm, q, args.steps, sync=False)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    st = P.last_stats3(ctx, grid)
    if st["nonphys"] or st["steps"] != args.steps:
        raise SystemExit(f"bench run failed: {st}")
    value = cells * 3 * args.steps / (gpu_ms / 1e3) / 1e9
    launch_ms = gpu_ms / (3 * args.steps)
    bytes_per_launch = cells * sum(BYTES_PER_CELL_STAGE_3D.values()) / 3.0
    achieved = bytes_per_launch / (launch_ms / 1e3) / 1e9
    traffic = measured_traffic(args.workload, args.precision)
    valu = measured_valu(args.workload, args.precision)
    alu = None
    if valu is not None:
        lane_rate = valu * cells / (launch_ms / 1e3)
        alu = {"bound": "alu", "achieved": round(lane_rate / 1e12, 3), "peak": round(PEAK_VALU_LANE_INSTR / 1e12, 3),
               "unit": "T VALU lane-instr/s", "frac": round(lane_rate / PEAK_VALU_LANE_INSTR, 4),
               "valu_lane_instr_per_cell_stage": valu}
    kform3 = "p" if P.SHAPES3[shape].endswith("p") else ("z" if "z" in P.SHAPES3[shape] else "")
    out = {
        "metric": "Gcell-updates/s per RK stage",
        "value": round(value, 4),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(gpu_ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 0 else "f32-flux/f64-state",
        "data": "synthetic",
        "config": {
            "workload": f"3-D low-Mach vortex {n}x{n}x{nz} (extruded along a periodic z, seeded w and "
                        "+-1e-6 checkerboard), M=0.01, FP64 state, MUSCL-minmod + SSP-RK3, Roe-AM (nine-face "
                        "detector, eps1=1, eps2=0.05), CFL 0.4",
            "cells": cells,
            "stages_per_step": 3,
            "tile_shape": P.SHAPES3[shape],
            "wall_s": round(wall, 4),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 2),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 5),
            "traffic": traffic,
            "traffic_frac": round(traffic / (launch_ms / 1e3) / 1e9 / PEAK_HBM_GBS, 5) if traffic else None,
            "alu": alu,
            "kernel": "k_stage3%s<order 2, FP%s, %s>" % (kform3, "64" if args.precision == 0 else "32-coef",
                                                         P.SHAPES3[shape]),
            "kernel_grid": f"{n}x{n}x{nz}",
            "launch_ms": round(launch_ms, 6),
            "timed_region_launches": 3 * args.steps,
            "algorithmic_bytes_per_launch": bytes_per_launch,
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_3d(case, args.cpu_sample_steps)
    print(json.dumps(out), flush=True)


def summarize_counters(args):
    """Write a counter summary for profiles/ from rocprofv3 --pmc CSV output
    (counter_collection.csv of the runs named by --pmc-csv): HBM bytes per
    stage-kernel launch from a FETCH_SIZE and a WRITE_SIZE pass, each scaled by
    what the counter reads for the run's plain 256 MiB copy, or the VALU work
    per cell-stage from an SQ pass.  Prints the summary; the caller saves it."""
    import csv
    import collections

    def load(path):
        per = collections.defaultdict(lambda: collections.defaultdict(float))
        names = {}
        for r in csv.DictReader(open(path)):
            key = r["Dispatch_Id"]
            per[key][r["Counter_Name"]] += float(r["Counter_Value"])
            names[key] = r["Kernel_Name"]
        return per, names

    cmd = args.pmc_command or "(command not given)"
    source_hash = kernel_source_hash(KERNEL_SOURCES_3D if is_3d(args.workload) else KERNEL_SOURCES)
    lines = []
    if args.pmc_kind == "traffic":
        lines.append(f"# HBM traffic per stage-kernel launch, {args.workload} (rocprofv3 --pmc, one pass per counter)")
        out = {}
        for path, ctr, what in zip(args.pmc_csv, ("FETCH_SIZE", "WRITE_SIZE"), ("read", "written")):
            lines.append(f"# {ctr} pass: {cmd.replace('<COUNTER>', ctr)}")
            per, names = load(path)
            stage = [per[k][ctr] for k in per if "k_stage" in names[k]]
            copies = [per[k][ctr] for k in per if "copy" in names[k].lower() and "k_stage" not in names[k]]
            kname = next(names[k] for k in per if "k_stage" in names[k])
            copy_kib = max(copies)
            scale = (256 << 20) / 1024.0 / copy_kib
            kib = sum(stage) / len(stage)
            c = ctr.lower()
            out[c] = (kib, len(stage), copy_kib, scale, kib * 1024 * scale)
        lines.append("# counters are KiB per dispatch; each is scaled by what it reads for a plain copy of 268435456 B")
        lines.append(f"kernel_source_hash {source_hash}")
        lines.append(f"kernel {kname.replace(' ', '')}")
        for c, (kib, n, ck, sc, b) in out.items():
            lines += [f"{c}_kib_per_dispatch {kib:.1f}", f"{c}_dispatches {n}", f"{c}_copy_kib {ck:.1f}",
                      f"{c}_scale {sc:.4f}", f"{c}_bytes_per_launch {b:.0f}"]
        lines.append(f"hbm_bytes_per_launch {out['fetch_size'][4] + out['write_size'][4]:.0f}")
    else:
        lines.append(f"# VALU work of the stage kernel per launch, {args.workload} (rocprofv3 --pmc, SQ block, whole-GPU sums)")
        lines.append(f"# command: {cmd}")
        lines.append("# SQ_INSTS_VALU counts wave64 instructions; x 64 / cells = lane-instructions per cell-stage")
        lines.append("# valu_busy_fraction = SQ_ACTIVE_INST_VALU / SQ_BUSY_CU_CYCLES")
        per, names = load(args.pmc_csv[0])
        keys = [k for k in per if "k_stage" in names[k]]
        tot = collections.defaultdict(float)
        for k in keys:
            for c, v in per[k].items():
                tot[c] += v
        n = len(keys)
        lines.append(f"kernel_source_hash {source_hash}")
        lines.append(f"kernel {names[keys[0]].replace(' ', '')}")
        lines.append(f"dispatches {n}")
        lines.append(f"cells {args.pmc_cells}")
        for c in sorted(tot):
            lines.append(f"{c.lower()}_per_dispatch {tot[c] / n:.0f}")
        lines.append(f"valu_lane_instr_per_cell_stage {tot['SQ_INSTS_VALU'] / n * 64 / args.pmc_cells:.1f}")
        if tot.get("SQ_BUSY_CU_CYCLES"):
            lines.append(f"valu_busy_fraction {tot['SQ_ACTIVE_INST_VALU'] / tot['SQ_BUSY_CU_CYCLES']:.3f}")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed bench steps: whole batches for batch256 (default 10), time steps for the "
                         "single-grid workloads (default 1000)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed bench steps before them (default 2 batches, or 50 time steps)")
    ap.add_argument("--spin-up-s", type=float, default=2.0,
                    help="seconds of the workload's own untimed GPU work before the warm-up steps, "
                         "so that the timed region runs at sustained clocks (0: none)")
    ap.add_argument("--workload", default="batch256",
                    help="batch256 (fourth configuration, the default line: 256 grids, 200 steps each, one "
                         "bench step = the whole batch), vortex256pair (the low-Mach vortex at both Mach "
                         "numbers, batched), vortexN (one N x N grid), serve (fifth configuration), "
                         "vortex3dNxNZ (one 3-D N x N x NZ grid), sod and oddeven (first and third "
                         "configurations, each run to its end time)")
    ap.add_argument("--precision", type=int, default=None, choices=[0, 1],
                    help="0 FP64, 1 FP32 coefficients (default: 0; batch256 defaults to 1)")
    ap.add_argument("--order", type=int, default=None, choices=[1, 2],
                    help="override the reconstruction order of the vortex workloads (roofline sweep)")
    ap.add_argument("--eps1", type=float, default=None, choices=[0.0, 1.0],
                    help="override eps1 of the vortex workloads (roofline sweep)")
    ap.add_argument("--time-scheme", type=int, default=None, choices=[0, 1, 2],
                    help="override the time scheme of the vortex workloads (counter runs only: the bench's "
                         "rates assume three stages per step)")
    ap.add_argument("--tile-shape", type=int, default=-1,
                    help="stage-kernel tile shape index for the vortex workloads (-1: autotune)")
    ap.add_argument("--batch-grids", type=int, default=256)
    ap.add_argument("--batch-persistent", action="store_true",
                    help="batch256: persistent batched stage kernels instead of one workgroup per tile")
    ap.add_argument("--no-extra-legs", action="store_true",
                    help="batch256: only the headline batch (no FP64 batch, one-at-a-time or 2048^2 legs)")
    ap.add_argument("--single-steps", type=int, default=100,
                    help="batch256: SSP-RK3 steps of the single-grid FP64 2048^2 leg")
    ap.add_argument("--rates", default="5,10,20")
    ap.add_argument("--duration", type=float, default=10.0)
    ap.add_argument("--serve-graph-iters", type=int, default=8)
    ap.add_argument("--split-cells", type=int, default=512 * 512,
                    help="serve: requests below this many cells go to the batched lane, larger ones to the "
                         "one-at-a-time lane")
    ap.add_argument("--serve-policy", type=int, default=0, choices=[0, 1],
                    help="admission order of queued requests: 0 FIFO, 1 shortest first (cells x steps)")
    ap.add_argument("--arena-gb", type=int, default=48)
    ap.add_argument("--profile-steps", type=int, default=100,
                    help="steps timed kernel by kernel with HIP events for the roofline object")
    ap.add_argument("--cpu-sample-steps", type=int, default=1000,
                    help="steps of each grid the oracle runs on all host threads (one thread runs at most 50)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--counter-run", action="store_true",
                    help="for rocprofv3 --pmc: only --profile-steps steps of directly launched stage "
                         "kernels, then a plain 256 MiB device copy as the counter reference; no timing")
    ap.add_argument("--summarize-pmc", dest="pmc_kind", choices=["traffic", "valu"], default=None,
                    help="no run: print a profiles/ counter summary from rocprofv3 CSV files (--pmc-csv)")
    ap.add_argument("--pmc-csv", nargs="+", default=[],
                    help="counter_collection.csv of the FETCH_SIZE then WRITE_SIZE passes (traffic), or of the SQ pass")
    ap.add_argument("--pmc-cells", type=int, default=0, help="cells per stage launch (valu summary)")
    ap.add_argument("--pmc-command", default="", help="the rocprofv3 command, <COUNTER> for the counter name")
    args = ap.parse_args()
    if args.pmc_kind:
        return summarize_counters(args)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the Roe-AM step here is a single-GPU build "
              "(multi-GPU sharding is described, not built). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    batch_like = args.workload == "batch256"
    if args.steps is None:
        args.steps = 10 if batch_like else 1000
    if args.warmup is None:
        args.warmup = 2 if batch_like else 50
    if args.counter_run:
        args.spin_up_s = 0.0  # counters do not depend on clocks
    # half the spin-up before anything else (the tile-shape autotuner then times
    # its candidates at sustained clocks), half with the workload's own work
    # right before its warm-up steps
    args.spin_up_s /= 2.0
    if args.spin_up_s > 0:
        spin_up_generic(args.spin_up_s)

    if args.workload == "batch256":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload in ("sod", "oddeven"):
        return bench_to_t_end(args)
    if args.precision is None:
        args.precision = 0
    if is_3d(args.workload):
        if args.cpu_sample_steps == 1000:
            args.cpu_sample_steps = 5
        return bench_3d(args)

    import torch
    import paper_1711_09272_amd as P

    if args.time_scheme is not None and not args.counter_run:
        raise SystemExit("--time-scheme is for counter runs (--counter-run)")
    cases, batched = make_cases(args.workload, args.precision, args.order, args.eps1, args.time_scheme)
    cells = sum(c.nx * c.ny for c in cases)
    ctx = P.Context(0)
    grids = [P.Grid.from_case(ctx, c) for c in cases]
    if args.tile_shape >= 0:
        for g in grids:
            g.set_tile_shape(args.tile_shape)
    case, grid = cases[0], grids[0]
    q = grid.to_device(case.q0)
    prm = case.params
    stream = torch.cuda.current_stream()

    if args.counter_run:
        if batched:
            P.step(ctx, grid, prm, grid.to_device(case.q0), 0)  # tile-shape tuning, as in the timed run
            P.batch_reserve(ctx, sum(g.footprint() for g in grids) + (1 << 20))
            profile_batch(ctx, grids, cases, args.profile_steps)
        else:
            P.profile_step(ctx, grid, prm, q, args.profile_steps)
        src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")  # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"counter_run": args.workload, "cells": cells,
                          "profile_steps": args.profile_steps, "copy_bytes": src.numel() * 8,
                          "tile_shape": grid.tile_shape(prm)}), flush=True)
        return

    if batched:
        gpu_ms, wall = timed_batch(ctx, grids, cases, args.steps, args.warmup, stream, args.spin_up_s)
    else:
        q_spin = grid.to_device(case.q0)
        spin_up(lambda: P.step(ctx, grid, prm, q_spin, 50, sync=True), args.spin_up_s)
        del q_spin
        # warmup (also tunes the tile shape and captures the step graphs)
        P.step(ctx, grid, prm, q, args.warmup, sync=True)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        P.step(ctx, grid, prm, q, args.steps, t0=0.0, t_end=0.0, sync=False)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        gpu_ms = ev0.elapsed_time(ev1)
        st = P.last_stats(ctx, grid)
        if st["nonphys"] or st["steps"] != args.steps:
            raise SystemExit(f"bench run failed: {st}")
    ms_per_step = gpu_ms / args.steps
    value = cells * 3 * args.steps / (gpu_ms / 1e3) / 1e9

    # roofline of the stage kernel that ran: HIP events around every stage
    # launch, on the library's stream
    if batched:
        stage_ms, launches = profile_batch(ctx, grids, cases, args.profile_steps)
        kname = "k_stage_batch"
        kgrid = " + ".join(f"{c.nx}x{c.ny}" for c in cases)
    else:
        stage_ms, launches = P.profile_step(ctx, grid, prm, q, args.profile_steps)
        kname = "k_stage_single"
        kgrid = f"{case.nx}x{case.ny}"
    shape = grid.tile_shape(prm)
    # average stage-launch duration over the timed region: its GPU time over
    # its stage launches (inter-kernel gaps and the batch engine's status
    # kernels count against the kernel, so this errs low); the event-bracketed
    # per-launch times above overstate kernels of ~10 us by the events' own cost
    launch_ms = gpu_ms / (3 * args.steps)
    bytes_per_launch = cells * sum(BYTES_PER_CELL_STAGE.values()) / 3.0
    achieved = bytes_per_launch / (launch_ms / 1e3) / 1e9
    # counter summaries are taken on the workload as configured; not for overridden variants
    overridden = args.order is not None or args.eps1 is not None
    traffic = None if overridden else measured_traffic(args.workload, args.precision)
    valu = None if overridden else measured_valu(args.workload, args.precision)
    alu = None
    if valu is not None:
        lane_rate = valu * cells / (launch_ms / 1e3)
        alu = {"bound": "alu", "achieved": round(lane_rate / 1e12, 3), "peak": round(PEAK_VALU_LANE_INSTR / 1e12, 3),
               "unit": "T VALU lane-instr/s", "frac": round(lane_rate / PEAK_VALU_LANE_INSTR, 4),
               "valu_lane_instr_per_cell_stage": valu}
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 2),
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": round(achieved / PEAK_HBM_GBS, 5),
        "traffic": traffic,
        "traffic_frac": round(traffic / (launch_ms / 1e3) / 1e9 / PEAK_HBM_GBS, 5) if traffic else None,
        "alu": alu,
        "kernel": "%s<order %d, FP%s, uniform, %s>" % (kname, prm["order"], "64" if args.precision == 0 else "32-coef",
                                                      P.SHAPES[shape] if shape >= 0 else "?"),
        "kernel_grid": kgrid,
        "launch_ms": round(launch_ms, 6),
        "timed_region_launches": 3 * args.steps,
        "event_bracketed_stage_ms": [round(x, 5) for x in stage_ms[:3]],
        "event_bracketed_launches": launches,
        "algorithmic_bytes_per_launch": bytes_per_launch,
    }

    out = {
        "metric": "Gcell-updates/s per RK stage",
        "value": round(value, 4),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 0 else "f32-flux/f64-state",
        "data": "synthetic",
        "config": {
            "workload": ("low-Mach isentropic vortex, two 256x256 periodic grids (M=0.01 and M=0.001) "
                         "advanced together as one batch" if batched else
                         f"low-Mach isentropic vortex {case.nx}x{case.ny} periodic, M=0.01")
                        + ", FP64 state, %s + SSP-RK3, Roe-AM (detector, eps1=%g, eps2=0.05), CFL 0.4"
                        % ("MUSCL-minmod" if prm["order"] == 2 else "first order", prm["eps1"]),
            "cells": cells,
            "grids": len(cases),
            "stages_per_step": 3,
            "tile_shape": P.SHAPES[shape] if shape >= 0 else None,
            "wall_s": round(wall, 4),
        },
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cases, args.cpu_sample_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
