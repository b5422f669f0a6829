#!/usr/bin/env python
"""Throughput of the Roe-AM step on one MI355X: Gcell-updates/s per RK stage.

Workload (default): the low-Mach isentropic vortex on a 256 x 256 periodic
grid, free-stream Mach 0.01, FP64, MUSCL-minmod + SSP-RK3, full Roe-AM
(detector on, eps1 = 1, eps2 = 0.05), CFL 0.4 with the c / sqrt(theta)
time-step rule; seeded +-1e-6 pressure checkerboard.  One bench step is one
SSP-RK3 time step (three fused stage kernels plus the on-device dt kernel) of
the whole grid, launched from captured HIP graphs.  Inputs are resident in
HBM before the timed region.

Prints one JSON line.  Extra legs: the roofline of the stage kernel (HIP
events around each stage launch), and the CPU oracle on a bounded sample.
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


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1711_09272_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per stage launch from committed rocprofv3 counter summaries,
    or None when missing or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"stage_kernel_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        parts = line.split()
        if len(parts) >= 2 and not line.startswith("#"):
            vals[parts[0]] = parts[1]
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def make_case(workload: str, precision: int):
    import workloads
    if workload == "vortex256":
        case = workloads.vortex(256, 0.01)
    elif workload.startswith("vortex"):
        n = int(workload[len("vortex"):])
        case = workloads.vortex(n, 0.01)
    else:
        raise SystemExit(f"unknown workload {workload}")
    case.params["precision"] = precision
    return case


def cpu_baseline(case, sample_steps: int):
    import oracle
    t0 = time.perf_counter()
    _, st = oracle.run(case, nsteps=sample_steps)
    dt = time.perf_counter() - t0
    cells = case.nx * case.ny
    return {
        "value": cells * 3 * st["steps"] / dt / 1e9,
        "unit": "Gcell-updates/s per RK stage",
        "cores": 1,
        "kind": "oracle",
        "sample": f"first {st['steps']} SSP-RK3 steps of the same {case.nx}x{case.ny} case "
                  f"({cells * 3 * st['steps']} cell-stage updates, {dt:.1f} s, single thread)",
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="vortex256")
    ap.add_argument("--precision", type=int, default=0, choices=[0, 1])
    ap.add_argument("--profile-steps", type=int, default=100,
                    help="steps timed kernel by kernel with HIP events for the roofline object")
    ap.add_argument("--cpu-sample-steps", type=int, default=150)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--counter-run", action="store_true",
                    help="for rocprofv3 --pmc: only --profile-steps steps of directly launched stage "
                         "kernels, then a plain 256 MiB device copy as the counter reference; no timing")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the Roe-AM step here is a single-GPU build "
              "(multi-GPU sharding is described, not built). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1711_09272_amd as P

    case = make_case(args.workload, args.precision)
    cells = case.nx * case.ny
    ctx = P.Context(0)
    grid = P.Grid.from_case(ctx, case)
    q = grid.to_device(case.q0)
    prm = case.params
    stream = torch.cuda.current_stream()

    if args.counter_run:
        P.profile_step(ctx, grid, prm, q, args.profile_steps)
        src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")  # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"counter_run": args.workload, "cells": cells, "profile_steps": args.profile_steps,
                          "copy_bytes": src.numel() * 8, "tile_shape": grid.tile_shape(prm)}), flush=True)
        return

    # warmup (also captures the step graphs)
    P.step(ctx, grid, prm, q, args.warmup, sync=True)
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
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
    shape = grid.tile_shape(prm)
    value = cells * 3 * args.steps / (gpu_ms / 1e3) / 1e9

    # roofline of the stage kernel: HIP events around every stage launch
    stage_ms, launches = P.profile_step(ctx, grid, prm, q, args.profile_steps)
    mean_ms = sum(stage_ms) / 3.0
    bytes_per_launch = cells * sum(BYTES_PER_CELL_STAGE.values()) / 3.0
    achieved = bytes_per_launch / (mean_ms / 1e3) / 1e9
    traffic = measured_traffic(args.workload)
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 2),
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": round(achieved / PEAK_HBM_GBS, 5),
        "traffic": traffic,
        "kernel": "k_stage_single<2,%d>" % args.precision,
        "stage_ms": [round(x, 5) for x in stage_ms],
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
            "workload": f"low-Mach isentropic vortex {case.nx}x{case.ny} periodic, M=0.01, "
                        "MUSCL-minmod + SSP-RK3, Roe-AM (detector, eps1=1, eps2=0.05), CFL 0.4",
            "cells": cells,
            "stages_per_step": 3,
            "tile_shape": ["32x15", "16x15", "8x7"][shape] if shape >= 0 else None,
            "wall_s": round(wall, 4),
        },
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_sample_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
