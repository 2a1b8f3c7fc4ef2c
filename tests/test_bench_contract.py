"""bench.py outside the GPU: the single-GPU contract and the gating of its
measured traffic figures on the kernel sources."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    lines = [x for x in r.stdout.splitlines() if x.strip()]
    assert len(lines) == 1
    msg = json.loads(lines[0])
    assert "one GPU" in msg["error"]


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_fields_follow_the_kernel_sources(tmp_path, monkeypatch):
    """The roofline traffic figures come from the committed counter summary
    only while it names the current kernel sources; otherwise they are null."""
    b = _bench_module()
    walk = tmp_path / "walk.hip"
    spmv = tmp_path / "spmv.hip"
    layout = tmp_path / "layout.h"  # shared by both kernels
    walk.write_text("// walk kernel v1\n")
    spmv.write_text("// spmv kernel v1\n")
    layout.write_text("// records v1\n")
    walk_src, spmv_src = [str(walk), str(layout)], [str(spmv), str(layout)]
    counters = tmp_path / "counters.md"
    counters.write_text(
        "| kernel | dispatches | FETCH | WRITE | calibrated bytes / launch | hit |\n"
        "| void spmv_pull_kernel<long, FwdGather, FwdEpi> | 87 | 1.0 | 2.0 | 1.5e+08 | 0.9 |\n\n"
        f"    kernel_source_sha256_16: {b.source_hash(walk_src)}\n"
        "    hbm_bytes_per_launch: 1.25e+12\n"
        f"    spmv_source_sha256_16: {b.source_hash(spmv_src)}\n")
    monkeypatch.setattr(b, "COUNTERS", str(counters))
    monkeypatch.setattr(b, "WALK_SOURCE", walk_src)
    monkeypatch.setattr(b, "SPMV_SOURCE", spmv_src)
    assert b.measured_traffic() == 1.25e12
    assert b.measured_spmv_traffic() == 1.5e8
    walk.write_text("// walk kernel v2\n")
    assert b.measured_traffic() is None
    assert b.measured_spmv_traffic() == 1.5e8
    spmv.write_text("// spmv kernel v2\n")
    assert b.measured_spmv_traffic() is None
    # a change to a layout header both kernels include voids both figures
    walk.write_text("// walk kernel v1\n")
    spmv.write_text("// spmv kernel v1\n")
    assert b.measured_traffic() == 1.25e12 and b.measured_spmv_traffic() == 1.5e8
    layout.write_text("// records v2\n")
    assert b.measured_traffic() is None and b.measured_spmv_traffic() is None
    monkeypatch.setattr(b, "COUNTERS", str(tmp_path / "missing.md"))
    assert b.measured_traffic() is None and b.measured_spmv_traffic() is None

