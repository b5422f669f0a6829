"""Build the gfx950 shared library libroeam.so in-tree with hipcc.

Usage: python -m paper_1711_09272_amd.build  (or build() from Python).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libroeam.so")
SOURCES = ["roeam_kernels.hip", "roeam_kernels_sc.hip", "roeam_norms.hip", "roeam_runtime.hip", "roeam_batch.hip",
           "roeam_batch_kernels.hip", "roeam_kernels3d.hip", "roeam_kernels3d_sc.hip", "roeam_runtime3d.hip"]
HEADERS = ["roeam_device.hpp", "roeam_internal.hpp", "roeam_stage.hpp", "roeam_stage2d.hpp", "roeam_device3d.hpp",
           "roeam_stage3d.hpp", "roeam_host.hpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # no packed FP32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose: bool = False, extra_flags=None) -> str:
    """Compile every source to an object in parallel (one hipcc per file), then
    link the shared library; the objects live in a build folder beside the
    package sources."""
    from concurrent.futures import ThreadPoolExecutor
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    common = [hipcc] + HIPCC_FLAGS + list(extra_flags or []) + ["-I", os.path.join(ROOT, "include"), "-I", CSRC]

    def compile_one(src):
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [c for c in common if c != "-shared"] + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        return obj, subprocess.run(cmd, capture_output=True, text=True)

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        results = list(ex.map(compile_one, sources()))
    for obj, res in results:
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError(f"hipcc failed compiling {os.path.basename(obj)[:-2]}")
    tmp = LIB + ".tmp"
    cmd = common + ["-o", tmp] + [obj for obj, _ in results]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking libroeam.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
