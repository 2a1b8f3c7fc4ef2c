"""Oracle passes over plain CSR arrays for graphs of a billion edges and more
(test infrastructure).

The sparse-matrix oracle (graph.py, exactsim.py) is the reference; this
module computes the same quantities with C loops (linear.c) so that the
largest workloads can be checked.  Its forward levels equal
exactsim.forward_levels bit for bit and its back-accumulation equals
exactsim.back_accumulate to rounding; the tests pin both on small graphs.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_lib = None


def _load():
    global _lib
    if _lib is None:
        from . import build as _b
        if not os.path.exists(_b.LINEAR_LIB):
            _b.build_linear(force=False)
        lib = ctypes.CDLL(_b.LINEAR_LIB)
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        lib.oracle_in_csr.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp]
        lib.oracle_in_csr.restype = ctypes.c_int
        lib.oracle_out_off.argtypes = [i64, i64, vp, vp]
        lib.oracle_out_off.restype = None
        lib.oracle_forward.argtypes = [i64, vp, vp, vp, i64, ctypes.c_double, ctypes.c_int, vp, vp]
        lib.oracle_forward.restype = ctypes.c_int
        lib.oracle_backward.argtypes = [i64, vp, vp, vp, vp, ctypes.c_int, vp, ctypes.c_double, vp]
        lib.oracle_backward.restype = ctypes.c_int
        _lib = lib
    return _lib


class CsrGraph:
    """n nodes and edges src -> dst (distinct, no self-loops, sorted by
    (src, dst), as the workload generators return them).  Exposes the
    attributes the walk and feature oracles read: n, m, din, dout, inv_din,
    in_off (int64), in_idx (int32, ascending source id per row)."""

    def __init__(self, n: int, src: np.ndarray, dst: np.ndarray):
        lib = _load()
        self.n = int(n)
        self.src = np.ascontiguousarray(src, dtype=np.int32)
        self.dst = np.ascontiguousarray(dst, dtype=np.int32)
        self.m = len(self.src)
        self.din = np.empty(n, dtype=np.int64)
        self.inv_din = np.empty(n, dtype=np.float64)
        self.in_off = np.empty(n + 1, dtype=np.int64)
        self.in_idx = np.empty(self.m, dtype=np.int32)
        rc = lib.oracle_in_csr(n, self.m, self.src.ctypes.data, self.dst.ctypes.data, self.din.ctypes.data,
                               self.inv_din.ctypes.data, self.in_off.ctypes.data, self.in_idx.ctypes.data)
        if rc != 0:
            raise ValueError("edges must be in range, distinct, without self-loops and sorted by (src, dst)")
        self.out_off = np.empty(n + 1, dtype=np.int64)
        lib.oracle_out_off(n, self.m, self.src.ctypes.data, self.out_off.ctypes.data)
        self.dout = np.diff(self.out_off)


def forward_levels(g: CsrGraph, u: int, c: float, L: int):
    """(levels[L+1, n], pi[n]) as exactsim.forward_levels computes them."""
    levels = np.empty((L + 1, g.n))
    pi = np.empty(g.n)
    rc = _load().oracle_forward(g.n, g.out_off.ctypes.data, g.dst.ctypes.data, g.inv_din.ctypes.data, u, c, L,
                                levels.ctypes.data, pi.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_forward: bad arguments")
    return levels, pi


def back_accumulate(g: CsrGraph, levels: np.ndarray, D: np.ndarray, c: float) -> np.ndarray:
    """s^L of Algorithm 1's back-accumulation, as exactsim.back_accumulate computes it."""
    levels = np.ascontiguousarray(levels, dtype=np.float64)
    D = np.ascontiguousarray(D, dtype=np.float64)
    L = levels.shape[0] - 1
    s = np.empty(g.n)
    rc = _load().oracle_backward(g.n, g.in_off.ctypes.data, g.in_idx.ctypes.data, g.inv_din.ctypes.data,
                                 levels.ctypes.data, L, D.ctypes.data, c, s.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_backward: bad arguments")
    return s
