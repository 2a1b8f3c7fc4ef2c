"""The C ABI library loads and exports every symbol its header declares;
host-only entry points work without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "exactsim.h")
LIB = os.path.join(ROOT, "paper_2004_03493_amd", "libexactsim.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(es_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_query_steps():
    syms = declared_symbols()
    for s in ("es_forward", "es_budget", "es_walk_pairs", "es_diag", "es_backward", "es_single_source", "es_topk"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2004_03493_amd import binding
    assert set(binding.SYMBOLS) == set(declared_symbols())


def test_host_constants_match_oracle_bitwise():
    from oracle import exactsim as ox
    from paper_2004_03493_amd import binding as es
    for c in (0.6, 0.8, 0.25):
        for eps in (1e-1, 1e-4, 1e-6, 3.3e-7):
            assert es.es_num_levels(c, eps) == ox.num_levels(c, eps)
            for n in (2, 2000, 1 << 20, 42_000_000):
                for r_scale in (1.0, 1e-5):
                    assert es.es_total_samples(n, c, eps, r_scale) == ox.total_samples(n, c, eps, r_scale)


def test_host_argument_errors():
    from paper_2004_03493_amd import binding as es
    for c, eps in ((0.0, 1e-3), (1.0, 1e-3), (0.6, 0.0), (0.6, 1.0), (float("nan"), 1e-3)):
        with pytest.raises(es.EsError) as e:
            es.es_num_levels(c, eps)
        assert e.value.status == es.ES_EINVAL
    with pytest.raises(es.EsError):
        es.es_total_samples(0, 0.6, 1e-3, 1.0)
    with pytest.raises(es.EsError):
        es.es_total_samples(10, 0.6, 1e-3, -1.0)


def test_status_strings():
    lib = ctypes.CDLL(LIB)
    lib.es_status_str.restype = ctypes.c_char_p
    for code in range(0, -7, -1):
        assert lib.es_status_str(code).startswith(b"ES_")


def test_context_without_device_reports_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is visible")
    lib = ctypes.CDLL(LIB)
    h = ctypes.c_void_p()
    lib.es_ctx_create.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    assert lib.es_ctx_create(0, None, ctypes.byref(h)) == -4  # ES_EDEVICE


def test_sparse_capacity_holds_the_pigeonhole_bound():
    # kept entries exceed theta and the levels' mass is at most 1 (plus the
    # forward pass's rounding), so the capacity is at least 1/theta entries
    # unless every entry of every level fits
    import math

    from oracle import exactsim as ox
    from paper_2004_03493_amd import binding as es
    for n, m in ((2000, 20000), (1 << 20, 16_000_000), (42_000_000, 1_400_000_000)):
        for c in (0.6, 0.8):
            for eps_s in (1e-2, 1e-4, 1e-6, 1e-9):
                L = ox.num_levels(c, 1e-6)
                cap = es.es_sparse_capacity(n, m, L, c, eps_s)
                theta = ox.sparse_threshold(c, eps_s)
                dense = (L + 1) * n
                assert cap <= dense
                assert cap >= min(dense, math.floor(1.0 / theta))
                slack = (L + 1) * (m + n) * 2.0 ** -62
                assert cap <= math.floor((1.0 + slack) / theta) + 1
    for bad in ((0.6, 0.0), (0.6, 1.0), (0.0, 1e-3), (1.0, 1e-3)):
        with pytest.raises(es.EsError):
            es.es_sparse_capacity(100, 100, 5, *bad)


def test_binding_structs_match_header_layout():
    # sizeof and every field offset of the option and statistics structs,
    # compiled from the header, against the binding's ctypes mirrors
    import shutil
    import subprocess

    from paper_2004_03493_amd import binding as es
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {"es_query_opts": es.QueryOpts, "es_stats": es.Stats, "es_batch_opts": es.BatchOpts}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "exactsim.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    out = os.path.join(ROOT, "_build", "abi")
    os.makedirs(out, exist_ok=True)
    src, exe = os.path.join(out, "layout.c"), os.path.join(out, "layout")
    with open(src, "w") as f:
        f.write("\n".join(lines) + "\n")
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
    got = {}
    for line in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n"):
        if line:
            cname, field, val = line.split()
            got[(cname, field)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for field, _ in py._fields_:
            assert got[(cname, field)] == getattr(py, field).offset, (cname, field)
