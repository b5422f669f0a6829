"""Host logic of bench.py, without a GPU: the one-GPU refusal, and the rule
that a committed rocprofv3 counter summary feeds the bench line only while its
kernel-source hash matches the current stage-kernel sources (2-D or 3-D set)."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_bench_refuses_more_than_one_gpu():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert p.returncode == 2 and "one GPU" in p.stdout + p.stderr


def test_kernel_source_hash_covers_the_stage_sources():
    B = load_bench()
    assert B.kernel_source_hash(B.KERNEL_SOURCES) != B.kernel_source_hash(B.KERNEL_SOURCES_3D)
    assert "roeam_stage2d.hpp" in B.KERNEL_SOURCES and "roeam_stage3d.hpp" in B.KERNEL_SOURCES_3D
    assert len(B.kernel_source_hash()) == 16


def test_counter_summaries_follow_the_kernel_source(tmp_path, monkeypatch):
    B = load_bench()
    monkeypatch.setattr(B, "ROOT", str(tmp_path))
    monkeypatch.setattr(B, "kernel_source_hash",
                        lambda sources=B.KERNEL_SOURCES: "h3d" if sources is B.KERNEL_SOURCES_3D else "h2d")
    prof = tmp_path / "profiles"
    prof.mkdir()

    def write(tag, kind, h, key, val):
        (prof / f"stage_kernel_{tag}_{kind}.txt").write_text(f"# comment {key} 0\nkernel_source_hash {h}\n{key} {val}\n")

    write("vortex2048", "traffic", "h2d", "hbm_bytes_per_launch", "3.5e8")
    write("vortex2048_fp32coef", "traffic", "stale", "hbm_bytes_per_launch", "3.5e8")
    write("vortex3d128x128", "valu", "h3d", "valu_lane_instr_per_cell_stage", "2286")
    write("vortex3d128x128_fp32coef", "valu", "h2d", "valu_lane_instr_per_cell_stage", "2212")
    assert B.measured_traffic("vortex2048", 0) == 3.5e8
    assert B.measured_traffic("vortex2048", 1) is None          # taken on another kernel source
    assert B.measured_valu("vortex3d128x128", 0) == 2286.0
    assert B.measured_valu("vortex3d128x128", 1) is None        # a 2-D hash on a 3-D summary
    assert B.measured_traffic("vortex256pair", 0) is None       # no summary
    assert B.measured_valu("vortex2048", 0) is None             # no such summary kind
