"""Native host code built with AddressSanitizer and UndefinedBehaviorSanitizer
and run on small and edge-case graphs: no invalid access, leak or undefined
operation.  Covered: the library's own host-side builders (edge packing, the
degree-ordered CSR layout, the SpMV row partition, the batched SpMM tiles),
and the test infrastructure's graph generators and oracle C passes."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1",
       "-fopenmp"]


@pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None, reason="gcc not available")
def test_generators_and_oracle_passes_are_sanitizer_clean():
    os.makedirs(OUT, exist_ok=True)
    objs = []
    for src in ("oracle/walks.c", "oracle/linear.c"):
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        subprocess.run(["gcc", "-std=c11", "-ffp-contract=off", *SAN, "-c", os.path.join(ROOT, src), "-o", obj],
                       check=True)
        objs.append(obj)
    exe = os.path.join(OUT, "sanitize_driver")
    subprocess.run(["g++", "-std=c++17", *SAN, os.path.join(ROOT, "tests", "native", "sanitize_driver.cpp"),
                    os.path.join(ROOT, "workloads", "graphgen.cpp"), *objs, "-o", exe, "-lm"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok"), r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_library_host_builders_are_sanitizer_clean():
    """es_host.cpp (the same source the library links) under the sanitizers:
    one node, no edges, duplicates and self-loops kept or dropped, rows over
    the SpMV's 8192 and the SpMM's 1024 cuts, 2.5e6 unsorted edges (several
    packing blocks, the parallel sort's merges), an out-of-range id; every
    CSR, partition and tile list checked against its invariants."""
    os.makedirs(OUT, exist_ok=True)
    csrc = os.path.join(ROOT, "paper_2004_03493_amd", "csrc")
    exe = os.path.join(OUT, "sanitize_host")
    flags = [f for f in SAN if f != "-fopenmp"] + ["-pthread"]
    subprocess.run(["g++", "-std=c++17", *flags, "-I", csrc, os.path.join(ROOT, "tests", "native", "sanitize_host.cpp"),
                    os.path.join(csrc, "es_host.cpp"), "-o", exe], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="3")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok"), r.stdout
