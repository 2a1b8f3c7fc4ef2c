"""Seeded synthetic inputs for ExactSim queries.

The paper evaluates on public power-law graphs (Section 4, Table 2), which
are not available here.  These generators stand in for them with the same
shapes: directed power-law graphs from a few thousand to tens of millions
of nodes, average degree 5-40, decay c = 0.6 (Section 4, "Methods and
parameters").

This module holds no ExactSim arithmetic.  It only produces edge lists,
source nodes and the parameter table of the standard workloads; the CPU
oracle and the HIP library both consume what it returns.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.cpp")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the generator library in place (g++ with OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.gg_rmat.argtypes = [ctypes.c_int32, ctypes.c_int64] + [ctypes.c_double] * 4 + [
            ctypes.c_uint64, i32p, i32p]
        lib.gg_rmat.restype = ctypes.c_int
        lib.gg_chung_lu.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64,
                                    i32p, i32p]
        lib.gg_chung_lu.restype = ctypes.c_int
        lib.gg_permutation.argtypes = [ctypes.c_int32, ctypes.c_uint64, i32p]
        lib.gg_permutation.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def rmat(n: int, m: int, seed: int, a=0.57, b=0.19, c=0.19, d=0.05):
    """Directed R-MAT graph: exactly m distinct edges, no self-loops, ids permuted.

    Returns (src, dst) int32 arrays sorted by (src, dst).
    """
    lib = _load()
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    rc = lib.gg_rmat(n, m, a, b, c, d, seed, _ptr(src), _ptr(dst))
    if rc != 0:
        raise ValueError(f"gg_rmat failed for n={n} m={m}")
    return src, dst


def chung_lu(n: int, m: int, seed: int, gamma: float = 2.1):
    """Directed Chung-Lu graph with aligned in/out weights (i+1)^(-1/(gamma-1)).

    Node 0 is the largest hub.  Returns (src, dst) int32 sorted by (src, dst).
    """
    lib = _load()
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    rc = lib.gg_chung_lu(n, m, gamma, seed, _ptr(src), _ptr(dst))
    if rc != 0:
        raise ValueError(f"gg_chung_lu failed for n={n} m={m}")
    return src, dst


def permutation(n: int, seed: int) -> np.ndarray:
    lib = _load()
    p = np.empty(n, dtype=np.int32)
    lib.gg_permutation(n, seed, _ptr(p))
    return p


def in_degrees(n: int, dst: np.ndarray) -> np.ndarray:
    return np.bincount(dst, minlength=n).astype(np.int64)


def pick_sources(n: int, dst: np.ndarray, count: int, seed: int, min_din: int = 2) -> np.ndarray:
    """`count` distinct source nodes, uniform over nodes with in-degree >= min_din.

    Nodes with in-degree 0 or 1 have trivial single-source answers, so the
    standard workloads draw their sources among the rest.
    """
    din = in_degrees(n, dst)
    pool = np.flatnonzero(din >= min_din)
    if len(pool) < count:
        raise ValueError("not enough eligible source nodes")
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(pool, size=count, replace=False)).astype(np.int32)


# ---------------------------------------------------------------------------
# The standard workloads.  Decay c = 0.6 as in the paper's experiments.
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    kind: str                  # "rmat" | "chung_lu" | "multi"
    n: int = 0
    m: int = 0
    c: float = 0.6
    eps: float = 1e-6
    seed_graph: int = 1
    seed_src: int = 2
    seed_walk: int = 3
    num_sources: int = 1
    fixed_sources: tuple = ()
    parts: list = field(default_factory=list)   # for kind == "multi"

    def graph(self):
        if self.kind == "rmat":
            return rmat(self.n, self.m, self.seed_graph)
        if self.kind == "chung_lu":
            return chung_lu(self.n, self.m, self.seed_graph)
        raise ValueError("multi-graph workload: use .graphs()")

    def sources(self, dst=None):
        if self.fixed_sources:
            return np.asarray(self.fixed_sources, dtype=np.int32)
        return pick_sources(self.n, dst, self.num_sources, self.seed_src)


CHUNG_LU_2K = Workload("chung_lu_n2000_m20000", "chung_lu", n=2000, m=20000, eps=1e-4,
                       seed_graph=11, seed_walk=13, fixed_sources=(0,))
RMAT_1M = Workload("rmat_n1048576_m16000000", "rmat", n=1 << 20, m=16_000_000, eps=1e-6,
                   seed_graph=21, seed_src=22, seed_walk=23, num_sources=8)
RMAT_4M8 = Workload("rmat_n4800000_m69000000_block64", "rmat", n=4_800_000, m=69_000_000,
                    eps=1e-6, seed_graph=31, seed_src=32, seed_walk=33, num_sources=64)
RMAT_42M = Workload("rmat_n42000000_m1400000000", "rmat", n=42_000_000, m=1_400_000_000,
                    eps=1e-6, seed_graph=51, seed_src=52, seed_walk=53, num_sources=8)


def uneven_parts(num_graphs: int = 12, n_lo: float = 1e4, n_hi: float = 2e6,
                 deg_lo: float = 5.0, deg_hi: float = 40.0, seed: int = 41):
    """Twelve graphs, n log-spaced 1e4..2e6, average degree linear 5..40,
    alternating R-MAT and Chung-Lu."""
    parts = []
    for g in range(num_graphs):
        t = g / (num_graphs - 1)
        n = int(round(n_lo * (n_hi / n_lo) ** t))
        deg = deg_lo + (deg_hi - deg_lo) * t
        m = int(round(n * deg))
        kind = "rmat" if g % 2 == 0 else "chung_lu"
        parts.append(Workload(f"part{g}", kind, n=n, m=m, seed_graph=seed * 100 + g))
    return parts


def uneven_source_counts(num_graphs: int, total: int, seed: int) -> np.ndarray:
    """Spread `total` sources over graphs Zipf(1)-unevenly, at least one each."""
    w = 1.0 / np.arange(1, num_graphs + 1)
    rng = np.random.Generator(np.random.PCG64(seed))
    order = rng.permutation(num_graphs)
    w = w[order]
    counts = np.ones(num_graphs, dtype=np.int64)
    rest = total - num_graphs
    extra = np.floor(rest * w / w.sum()).astype(np.int64)
    counts += extra
    left = total - counts.sum()
    frac = rest * w / w.sum() - extra
    for g in np.argsort(-frac)[:left]:
        counts[g] += 1
    return counts


UNEVEN_12 = Workload("uneven_12graphs_256src", "multi", eps=1e-6, seed_src=42, seed_walk=43,
                     num_sources=256, parts=uneven_parts())

WORKLOADS = {w.name: w for w in (CHUNG_LU_2K, RMAT_1M, RMAT_4M8, UNEVEN_12, RMAT_42M)}
