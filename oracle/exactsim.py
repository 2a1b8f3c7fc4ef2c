"""ExactSim estimator, step by step in the paper's order (test infrastructure).

Algorithm 1 (basic ExactSim) with the pi^2 allocation of Section 3.2, in
its own order:

  1. level count      L = ceil(log_{1/c}(2/eps))
  2. l-hop PPR        pi^0 = (1 - sqrt c) e_u;  pi^l = sqrt c P pi^(l-1);
                      pi = sum_l pi^l
  3. sample count     R = 6 ln n / ((1 - sqrt c)^4 eps^2)
  4. diagonal         R(k) = ceil(R pi(k)^2) pairs of sqrt(c)-walks for node
                      k; D^(k,k) is the fraction of pairs that do not meet
                      (Algorithm 2)
  5. back-accumulate  s^0 = D^ pi^L / (1 - sqrt c);
                      s^l = sqrt c P^T s^(l-1) + D^ pi^(L-l) / (1 - sqrt c)
  6. result           s^L

Readings where the text is ambiguous (each also listed in the design notes):

* L is found as the smallest l >= 0 with c^l <= eps/2, c^l formed by repeated
  float64 multiplication; that is the level count's ceiling without a float
  logarithm deciding an integer.
* ln is the natural logarithm (the bound behind R is Bernstein's, which is
  exponential).  R is kept in float64 and multiplied by an explicit
  ``r_scale`` (1 = the paper's R).
* Section 3.2 prints R(k) = R ceil(pi(k)^2/||pi||^2), which as typeset gives
  every touched node R samples; its proof (Lemma 3) uses
  rho(k) = ceil(R' pi(k)^2/||pi||^2)/R' with R' = R ||pi||^2.  Both readings
  agree on R(k) = ceil(R pi(k)^2), which is what is computed.
* Algorithm 3, its exact cases: a node without in-neighbours has D = 1 and a node
  with exactly one has D = 1 - c, exactly.  With ``exact_small_din`` those
  nodes get no samples and these values.
* Floating point decides integers here (the sample counts), so the forward
  pass fixes its rounding: every term pi^(l-1)(j)/d_in(j) is rounded once to
  the nearest multiple of 2^-62 (ties to even) and summed exactly in 64-bit
  integers; pi^l(i) = sqrt c * (acc * 2^-62).  The result differs from exact
  arithmetic by at most d_out(i) 2^-63 per entry and does not depend on the
  summation order.
* Sparse linearization (Section 3.2, Lemma 2) removes the stored entries
  pi^l(k) <= (1 - sqrt c)^2 eps_s.  The forward pass still propagates the full
  vectors and the budget uses the full pi(k); only the copy of the levels that
  the back-accumulation reads is sparse (``sparse_eps`` of ``query``).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from .graph import OracleGraph

FIX_SCALE = 2.0 ** 62
FIX_INV = 2.0 ** -62
TMAX = 4096


# ---------------------------------------------------------------------------
# Host constants
# ---------------------------------------------------------------------------

def num_levels(c: float, eps: float) -> int:
    """Smallest L >= 0 with c^L <= eps/2 (Algorithm 1, the level count)."""
    L = 0
    p = 1.0
    half = eps / 2.0
    while p > half:
        p = p * c
        L += 1
    return L


def total_samples(n: int, c: float, eps: float, r_scale: float = 1.0) -> float:
    """R = 6 ln n / ((1 - sqrt c)^4 eps^2), times r_scale (Algorithm 1, the sample count)."""
    sc = math.sqrt(c)
    om = 1.0 - sc
    om2 = om * om
    om4 = om2 * om2
    return 6.0 * math.log(n) / (om4 * (eps * eps)) * r_scale


def lifetime_thresholds(c: float) -> np.ndarray:
    """thr[t] = floor(c^t 2^64), t >= 1, while positive (thr[0] unused = 0)."""
    thr = [0]
    p = 1.0
    for _ in range(TMAX):
        p = p * c
        v = int(p * 18446744073709551616.0)
        if v == 0:
            break
        thr.append(min(v, (1 << 64) - 1))
    return np.array(thr, dtype=np.uint64)


# ---------------------------------------------------------------------------
# Step 2: l-hop PPR vectors (Algorithm 1)
# ---------------------------------------------------------------------------

def forward_levels(g: OracleGraph, u: int, c: float, L: int):
    """Return (pi_levels[L+1, n], pi[n]) in the fixed-point rounding above."""
    sc = math.sqrt(c)
    n = g.n
    levels = np.zeros((L + 1, n))
    levels[0, u] = 1.0 - sc
    pi = levels[0].copy()
    for l in range(1, L + 1):
        term = levels[l - 1] * g.inv_din                      # pi^(l-1)(j) / d_in(j)
        q = np.rint(term * FIX_SCALE).astype(np.int64)        # nearest multiple of 2^-62
        acc = g.A_int @ q                                     # exact sum over j in O(i)
        levels[l] = sc * (acc.astype(np.float64) * FIX_INV)
        pi = pi + levels[l]
    return levels, pi


# ---------------------------------------------------------------------------
# Step 3-4: sample budget (Algorithm 1, Section 3.2)
# ---------------------------------------------------------------------------

def budget(pi: np.ndarray, din: np.ndarray, R: float, exact_small_din: bool = True) -> np.ndarray:
    """R(k) = ceil(R * (pi(k) * pi(k))) as uint64 (two separate products)."""
    Rk = np.ceil(R * (pi * pi))
    if exact_small_din:
        Rk[din <= 1] = 0.0
    return Rk.astype(np.uint64)


def budget_pi(pi: np.ndarray, din: np.ndarray, R: float, exact_small_din: bool = True) -> np.ndarray:
    """Basic allocation of Algorithm 1: R(k) = ceil(R * pi(k))."""
    Rk = np.ceil(R * pi)
    if exact_small_din:
        Rk[din <= 1] = 0.0
    return Rk.astype(np.uint64)


_walk_lib = None


def _walks():
    global _walk_lib
    if _walk_lib is None:
        from . import build as _b
        if not os.path.exists(_b.LIB):
            _b.build(force=False)
        lib = ctypes.CDLL(_b.LIB)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.oracle_philox4x64_10.argtypes = [u64p, u64p, u64p]
        lib.oracle_philox4x64_10.restype = None
        lib.oracle_mulhi64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.oracle_mulhi64.restype = ctypes.c_uint64
        lib.oracle_lifetime_table.argtypes = [ctypes.c_double, u64p, ctypes.c_int]
        lib.oracle_lifetime_table.restype = ctypes.c_int
        lib.oracle_walk_pair.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, u64p, ctypes.c_int,
                                         ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int]
        lib.oracle_walk_pair.restype = ctypes.c_int
        lib.oracle_walk_counts.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double,
                                           ctypes.c_void_p, ctypes.c_int]
        lib.oracle_walk_counts.restype = ctypes.c_int
        lib.oracle_max_threads.restype = ctypes.c_int
        _walk_lib = lib
    return _walk_lib


def philox4x64_10(counter, key) -> np.ndarray:
    lib = _walks()
    ctr = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.oracle_philox4x64_10(ctr.ctypes.data_as(u64p), k.ctypes.data_as(u64p), out.ctypes.data_as(u64p))
    return out


def mulhi64(w: int, d: int) -> int:
    return int(_walks().oracle_mulhi64(w, d))


def c_lifetime_thresholds(c: float) -> np.ndarray:
    lib = _walks()
    buf = np.zeros(TMAX + 1, dtype=np.uint64)
    cnt = lib.oracle_lifetime_table(c, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), TMAX + 1)
    return buf[: cnt + 1]


def walk_pair(g: OracleGraph, seed: int, c: float, k: int, r: int, nonstop: int = 0) -> int:
    lib = _walks()
    thr = c_lifetime_thresholds(c)
    return int(lib.oracle_walk_pair(g.in_off.ctypes.data, g.in_idx.ctypes.data, seed,
                                    thr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), len(thr) - 1, k, r,
                                    nonstop))


def walk_counts(g: OracleGraph, Rk: np.ndarray, seed: int, c: float, threads: int = 0,
                r_begin: np.ndarray | None = None, nonstop: np.ndarray | None = None) -> np.ndarray:
    """M(k): meeting pairs among pairs r in [r_begin(k), R(k)) of each node (Algorithm 2);
    with nonstop(k) = l > 0, the non-stop pairs of Algorithm 3 (meetings after step l)."""
    lib = _walks()
    Rk = np.ascontiguousarray(Rk, dtype=np.uint64)
    M = np.zeros(g.n, dtype=np.uint64)
    rb = None if r_begin is None else np.ascontiguousarray(r_begin, dtype=np.uint64)
    ns = None if nonstop is None else np.ascontiguousarray(nonstop, dtype=np.int32)
    rc = lib.oracle_walk_counts(g.n, g.in_off.ctypes.data, g.in_idx.ctypes.data,
                                None if rb is None else rb.ctypes.data, Rk.ctypes.data,
                                None if ns is None else ns.ctypes.data, seed, c, M.ctypes.data, threads)
    if rc != 0:
        raise ValueError("oracle_walk_counts: bad arguments")
    return M


def max_threads() -> int:
    return int(_walks().oracle_max_threads())


# ---------------------------------------------------------------------------
# Step 4 (estimate) and step 5 (back-accumulation)
# ---------------------------------------------------------------------------

def diag_estimate(Rk: np.ndarray, M: np.ndarray, din: np.ndarray, c: float,
                  exact_small_din: bool = True) -> np.ndarray:
    """D^(k,k) = (R(k) - M(k)) / R(k)  (Algorithm 2, fraction of non-meeting pairs).

    Nodes with no samples get 1 (their pi is zero, so the value is never used),
    except the exact cases that open Algorithm 3."""
    D = np.ones(len(Rk))
    has = Rk > 0
    D[has] = (Rk[has] - M[has]).astype(np.float64) / Rk[has].astype(np.float64)
    if exact_small_din:
        D[din == 0] = 1.0
        D[din == 1] = 1.0 - c
    return D


def back_accumulate(g: OracleGraph, levels: np.ndarray, D: np.ndarray, c: float) -> np.ndarray:
    """s^L by the nested recursion of Algorithm 1's back-accumulation."""
    sc = math.sqrt(c)
    a = 1.0 / (1.0 - sc)
    L = levels.shape[0] - 1
    s = a * (D * levels[L])
    for l in range(1, L + 1):
        s = sc * (g.inv_din * (g.AT @ s)) + a * (D * levels[L - l])
    return s


# ---------------------------------------------------------------------------
# Sparse linearization (Section 3.2, Lemma 2)
# ---------------------------------------------------------------------------

def sparse_threshold(c: float, eps_s: float) -> float:
    """theta = (1 - sqrt c)^2 eps_s, the cut of sparse linearization: stored
    entries pi^l(k) <= theta are removed, which adds at most eps_s to every
    s(u, j) (Lemma 2) and leaves at most 1/theta entries over all levels (the
    levels' total mass is at most 1).  Evaluated as ((1 - sc) * (1 - sc)) *
    eps_s in float64."""
    sc = math.sqrt(c)
    return (1.0 - sc) * (1.0 - sc) * eps_s


def sparsify_levels(levels: np.ndarray, theta: float) -> np.ndarray:
    """The levels that sparse linearization keeps: every pi^l(k) <= theta set to zero.

    Reading: the forward pass itself propagates the full pi^(l-1) (so every
    kept entry is exact and each removed one is off by less than theta, the
    per-entry error Lemma 2's proof assumes); only the stored copy that the
    back-accumulation reads is sparse, and the sample budget uses the full
    pi(k) of the forward pass."""
    out = np.array(levels, dtype=np.float64, copy=True)
    out[out <= theta] = 0.0
    return out


def topk(s: np.ndarray, u: int, k: int):
    """k largest s(j), j != u, ties to the smaller id."""
    idx = np.arange(len(s))
    keep = idx != u
    order = np.lexsort((idx[keep], -s[keep]))
    sel = idx[keep][order[:k]]
    return sel.astype(np.int32), s[sel]


def query(g: OracleGraph, u: int, c: float, eps: float, seed: int, r_scale: float = 1.0,
          exact_small_din: bool = True, d_override: np.ndarray | None = None, alloc: str = "pi2",
          threads: int = 0, sparse_eps: float = 0.0) -> dict:
    """One ExactSim single-source query; returns every intermediate.

    ``sparse_eps`` > 0 runs the back-accumulation on the levels of sparse
    linearization with threshold sparse_threshold(c, sparse_eps)."""
    L = num_levels(c, eps)
    levels, pi = forward_levels(g, u, c, L)
    R = total_samples(g.n, c, eps, r_scale)
    if d_override is not None:
        Rk = np.zeros(g.n, dtype=np.uint64)
        M = np.zeros(g.n, dtype=np.uint64)
        D = np.asarray(d_override, dtype=np.float64)
    else:
        if alloc == "pi2":
            Rk = budget(pi, g.din, R, exact_small_din)
        elif alloc == "pi":
            Rk = budget_pi(pi, g.din, R, exact_small_din)
        else:
            raise ValueError(alloc)
        M = walk_counts(g, Rk, seed, c, threads)
        D = diag_estimate(Rk, M, g.din, c, exact_small_din)
    kept = levels
    if sparse_eps > 0.0:
        kept = sparsify_levels(levels, sparse_threshold(c, sparse_eps))
    s = back_accumulate(g, kept, D, c)
    return dict(L=L, R=R, levels=levels, kept=kept, pi=pi, Rk=Rk, M=M, D=D, s=s)
