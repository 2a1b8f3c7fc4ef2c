"""Local deterministic exploitation for D(k,k) (Section 3.2, Algorithm 3,
Lemma 4): test infrastructure.

Z_l(k, q) is the probability that two sqrt(c)-walks from v_k first meet at
v_q at their l-th step, Z_l(k) = sum_q Z_l(k, q), and
D(k,k) = 1 - sum_{l >= 1} Z_l(k).  With (P^T)^l(k, q) the probability that a
walk from v_k that never stops sits at v_q after l steps (each step to a
uniformly random in-neighbour; a walk at a node without in-neighbours is
lost), Lemma 4 gives

    Z_l(k, q) = c^l (P^T)^l(k, q)^2
                - sum_{l'=1}^{l-1} sum_{q'} c^l' (P^T)^l'(q', q)^2 Z_{l-l'}(k, q').

Algorithm 3 computes sum_{l <= l(k)} Z_l(k) exactly and estimates the rest
with pairs of walks that do not stop during their first l(k) steps and are
sqrt(c)-walks afterwards: a pair that meets after step l(k) without having
met before has probability c^-l(k) sum_{l > l(k)} Z_l(k), so

    D^(k,k) = (1 - sum_{l=1}^{l(k)} Z_l(k)) - c^l(k) * (M(k) / R'(k))

over R'(k) such pairs of which M(k) meet after step l(k).

The level l(k) comes from Algorithm 3's edge counter.  Round l (l = 0, 1,
...) first evaluates Z_l(k, .) and then extends transition tables by one
step: for l' = 0..l and every node q' with (P^T)^{l-l'}(k, q') > 0, the table
(P^T)^{l'}(q', .) becomes (P^T)^{l'+1}(q', .), one edge counted in E_k per
in-neighbour of every node in the table's support.  The exploitation stops
in the round where E_k reaches 2 R(k) / sqrt(c), and l(k) is that round.

Readings (the printed loop is open-ended and its tables are shared):
  * E_k counts every edge the loops traverse, also when an origin q' lies
    at several depths from v_k and its table is extended again; a table
    holds transition probabilities (extending it again does not add to
    them).
  * A round that traverses no edge ends the exploitation: no walk from v_k
    survives one more step, every first meeting has been counted, and l(k)
    is that round.
  * The caller caps the level: l(k) = min(l_printed(k), cap); the rounds
    after the cap are never counted.
  * The threshold test is the float64 comparison E >= (2 R(k)) / sqrt(c).
  * Nodes with R(k) = 0 take no samples and run no exploitation (l = 0).
  * R'(k) = R(k) as printed ("as_printed"), or R'(k) = ceil(R(k) c^l(k))
    ("reduced"): each pair then weighs c^l(k)/R'(k) <= 1/R(k) and its
    Bernoulli variance is at most 1/4, so the range and variance terms of
    the Bernstein bound behind Theorem 1 are no larger than with R(k) plain
    pairs.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import scipy.sparse as sp

MODE_OFF, MODE_AS_PRINTED, MODE_REDUCED = 0, 1, 2
DEFAULT_MAX_LEVEL = 3

_lib = None


def _load():
    global _lib
    if _lib is None:
        from . import build as _b
        if not os.path.exists(_b.LDE_LIB):
            _b.build_lde(force=False)
        lib = ctypes.CDLL(_b.LDE_LIB)
        vp = ctypes.c_void_p
        lib.lde_levels.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_int64, vp, vp, ctypes.c_int32, vp, vp]
        lib.lde_levels.restype = ctypes.c_int
        _lib = lib
    return _lib


# ---------------------------------------------------------------------------
# Lemma 4
# ---------------------------------------------------------------------------

def transition_rows(g, rows, m: int) -> sp.csr_matrix:
    """Rows `rows` of (P^T)^m as a sparse matrix (len(rows) x n)."""
    rows = np.asarray(rows, dtype=np.int64)
    out = sp.csr_matrix((np.ones(len(rows)), (np.arange(len(rows)), rows)), shape=(len(rows), g.n))
    for _ in range(m):
        out = sp.csr_matrix(out @ g.PT)
    return out


def first_meeting(g, k: int, c: float, L: int) -> np.ndarray:
    """Z_l(k) for l = 0..L (Z_0 = 0) by Lemma 4."""
    Z = np.zeros(L + 1)
    Zq = {}
    for l in range(1, L + 1):
        pk = transition_rows(g, [k], l)
        v = (c ** l) * pk.multiply(pk)
        for lp in range(1, l):
            prev = Zq[l - lp]
            if prev.nnz == 0:
                continue
            rows = transition_rows(g, prev.indices, lp)
            v = v - (c ** lp) * sp.csr_matrix(prev.data[None, :] @ rows.multiply(rows))
        Zq[l] = sp.csr_matrix(v)
        Z[l] = float(Zq[l].sum())
    return Z


def brute_first_meeting(g, k: int, c: float, L: int) -> np.ndarray:
    """Z_l(k) for l = 0..L by enumerating the joint positions of two
    independent sqrt(c)-walks that have not met yet (small graphs only)."""
    Z = np.zeros(L + 1)
    states = {(k, k): 1.0}
    for t in range(1, L + 1):
        nxt = {}
        for (x, y), p in states.items():
            nx, ny = g.in_neighbours(x), g.in_neighbours(y)
            if len(nx) == 0 or len(ny) == 0:
                continue
            pp = p * c / (len(nx) * len(ny))
            for a in nx:
                for b in ny:
                    if a == b:
                        Z[t] += pp
                    else:
                        nxt[(int(a), int(b))] = nxt.get((int(a), int(b)), 0.0) + pp
        states = nxt
    return Z


# ---------------------------------------------------------------------------
# Algorithm 3's deterministic part, as printed (small graphs)
# ---------------------------------------------------------------------------

def printed_exploitation(g, k: int, c: float, T: float, cap: int | None = None):
    """Run the deterministic part of Algorithm 3 for node k with edge budget
    T = 2 R(k) / sqrt(c): rounds of Z_l by Lemma 4 and table extensions with
    the edge counter E_k.  Returns (l(k), Z, costs): Z[l] = Z_l(k) for
    l = 0..l(k) and costs[l] the edges counted in round l (the last one up
    to the stop).  Pure Python dictionaries; for graphs of a few dozen
    nodes."""
    din = g.din

    def nbrs(v):
        return g.in_idx[g.in_off[v]:g.in_off[v + 1]]

    tab = {(k, 0): {k: 1.0}}    # tab[(q', j)] = {x: (P^T)^j(q', x)}
    Zq = {}                     # Zq[l] = {q: Z_l(k, q)}
    Z = []
    costs = []
    E = 0
    l = 0
    while True:
        # Z_l(k, q) for every q with (P^T)^l(k, q) != 0 (Lemma 4)
        cur = {}
        for q, p in tab[(k, l)].items():
            z = (c ** l) * p * p
            for lp in range(1, l):
                for q2, z2 in Zq[l - lp].items():
                    t = tab[(q2, lp)].get(q, 0.0)
                    z -= (c ** lp) * t * t * z2
            cur[q] = z
        Zq[l] = cur
        Z.append(sum(cur.values()) if l > 0 else 0.0)
        if cap is not None and l >= cap:
            return l, Z, costs
        # extend the tables one step, counting traversed edges
        cost = 0
        for lp in range(l + 1):
            for q2 in list(tab[(k, l - lp)].keys()):
                src = tab.setdefault((q2, lp), {q2: 1.0} if lp == 0 else None)
                nxt = {}
                for x, px in src.items():
                    for q in nbrs(x):
                        nxt[int(q)] = nxt.get(int(q), 0.0) + px / din[x]
                        cost += 1
                        if E + cost >= T:
                            costs.append(cost)
                            return l, Z, costs
                tab[(q2, lp + 1)] = nxt
        costs.append(cost)
        if cost == 0:
            return l, Z, costs
        E += cost
        l += 1


# ---------------------------------------------------------------------------
# The level rule on large graphs (C, oracle/lde_count.c)
# ---------------------------------------------------------------------------

def edge_budget(Rk: np.ndarray, c: float) -> np.ndarray:
    """2 R(k) / sqrt(c) in float64, in that order."""
    return (2.0 * np.asarray(Rk, dtype=np.uint64).astype(np.float64)) / math.sqrt(c)


def printed_levels(g, nodes, T, cap: int, with_costs: bool = False):
    """min(l_printed(k), cap) for k in nodes with edge budgets T (C loops
    over the graph's in-CSR); with_costs also returns the edges counted in
    each round [len(nodes), cap] (-1 for rounds not run)."""
    lib = _load()
    nodes = np.ascontiguousarray(nodes, dtype=np.int32)
    T = np.ascontiguousarray(T, dtype=np.float64)
    in_off = np.ascontiguousarray(g.in_off, dtype=np.int64)
    in_idx = np.ascontiguousarray(g.in_idx, dtype=np.int32)
    ell = np.zeros(len(nodes), dtype=np.int32)
    costs = np.zeros((len(nodes), max(cap, 1)), dtype=np.int64) if with_costs else None
    rc = lib.lde_levels(int(g.n), in_off.ctypes.data, in_idx.ctypes.data, len(nodes), nodes.ctypes.data,
                        T.ctypes.data, int(cap), ell.ctypes.data, costs.ctypes.data if with_costs else None)
    if rc != 0:
        raise ValueError("lde_levels: bad argument")
    return (ell, costs) if with_costs else ell


def c_power(c: float, l: int) -> float:
    """c^l by repeated float64 multiplication."""
    p = 1.0
    for _ in range(l):
        p = p * c
    return p


def plan(g, Rk: np.ndarray, c: float, mode: int, max_level: int = DEFAULT_MAX_LEVEL, zsum_nodes="all"):
    """(l(k) int32[n], sum_{l<=l(k)} Z_l(k) float64[n], R'(k) uint64[n]) for
    every node: l(k) = min(l_printed(k), max_level) where R(k) > 0, else 0.
    Z by Lemma 4: c/d_in(k) for l(k) = 1; for l(k) >= 2 only at the nodes
    of zsum_nodes ("all", or an array of ids; NaN elsewhere)."""
    n = g.n
    Rk = np.asarray(Rk, dtype=np.uint64)
    ell = np.zeros(n, dtype=np.int32)
    zsum = np.zeros(n)
    if mode == MODE_OFF:
        return ell, zsum, Rk.copy()
    act = np.flatnonzero(Rk > 0).astype(np.int32)
    ell[act] = printed_levels(g, act, edge_budget(Rk[act], c), max_level)
    one = ell == 1
    zsum[one] = c / g.din[one].astype(np.float64)
    deep = np.flatnonzero(ell >= 2)
    want = set(deep.tolist()) if isinstance(zsum_nodes, str) else set(int(x) for x in zsum_nodes)
    for k in deep:
        zsum[k] = float(first_meeting(g, int(k), c, int(ell[k]))[1:].sum()) if int(k) in want else np.nan
    if mode == MODE_REDUCED:
        cl = np.array([c_power(c, l) for l in range(int(ell.max(initial=0)) + 1)])
        R2 = np.ceil(Rk.astype(np.float64) * cl[ell]).astype(np.uint64)
        R2[Rk == 0] = 0
    else:
        R2 = Rk.copy()
    return ell, zsum, R2


def diag_estimate(Rk: np.ndarray, M: np.ndarray, ell: np.ndarray, zsum: np.ndarray, c: float, din: np.ndarray,
                  exact_small_din: bool = True) -> np.ndarray:
    """D^(k,k): (R - M)/R where l(k) = 0 (Algorithm 2), else
    (1 - sum Z) - c^l(k) (M / R) (Algorithm 3); the exact shortcuts that
    open Algorithm 3 for d_in <= 1."""
    n = len(Rk)
    D = np.ones(n)
    has = Rk > 0
    R = Rk.astype(np.float64)
    Mf = M.astype(np.float64)
    basic = has & (ell == 0)
    D[basic] = (Rk[basic] - M[basic]).astype(np.float64) / R[basic]
    lde = has & (ell > 0)
    cl = np.array([c_power(c, l) for l in range(int(ell.max(initial=0)) + 1)])
    D[lde] = (1.0 - zsum[lde]) - cl[ell[lde]] * (Mf[lde] / R[lde])
    if exact_small_din:
        D[din == 0] = 1.0
        D[din == 1] = 1.0 - c
    return D
