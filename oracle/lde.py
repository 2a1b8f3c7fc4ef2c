"""Local deterministic exploitation for D(k,k) (Section 3.3, Algorithm 3,
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

Readings (the loop nesting of Algorithm 3 is garbled in the text):
  * l(k) is the largest l <= l_max(k) whose deterministic work stays within
    the algorithm's bound 2 R(k) / sqrt(c); l(k) = 0 (plain Algorithm 2)
    when even level 1 exceeds it or R(k) = 0.  The work W_l(k) counts the
    in-walks of length <= l from v_k, E_l(k) = sum_{m <= l} (number of
    length-m in-walks); the third level's walks are charged at their GPU
    cost, W_3 = E_2 + level3_path_cost(n) (E_3 - E_2): each of them is two
    atomic updates of a node-sized array, about 2 walk steps when that
    array stays in cache and 24 when its updates go to HBM.
    l_max is 3 for the query source, whose pairs dominate the budget, and 1
    for every other node (Z_1(k) = c / d_in(k) is a closed form).
  * R'(k) = R(k) as printed ("as_printed"), or R'(k) = ceil(R(k) c^l(k))
    ("reduced"): each pair then weighs c^l(k)/R'(k) <= 1/R(k) and its
    Bernoulli variance is at most 1/4, so the range and variance terms of
    the Bernstein bound behind Theorem 1 are no larger than with R(k) plain
    pairs.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

MAX_SOURCE_LEVEL = 3
MODE_OFF, MODE_AS_PRINTED, MODE_REDUCED = 0, 1, 2


def level3_path_cost(n: int) -> int:
    """Work charged per three-step in-walk of the source's third exact level:
    2 walk steps when the node-sized accumulator (8n bytes) fits in 128 MiB
    of cache, 24 when it does not (measured on MI355X)."""
    return 2 if 8 * n <= 1 << 27 else 24


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


def edge_costs(g, k: int) -> tuple[int, int, int]:
    """(E_1, E_2, E_3): edges traversed by the deterministic part up to
    levels 1, 2, 3 (in-walks of length 1, 2, 3 from v_k, cumulated)."""
    din = g.din
    nb = g.in_idx[g.in_off[k]:g.in_off[k + 1]]
    e1 = int(len(nb))
    e2 = e1 + int(din[nb].sum())
    e3 = e2 + sum(int(din[g.in_idx[g.in_off[a]:g.in_off[a + 1]]].sum()) for a in nb)
    return e1, e2, e3


def c_power(c: float, l: int) -> float:
    """c^l by repeated float64 multiplication."""
    p = 1.0
    for _ in range(l):
        p = p * c
    return p


def plan(g, u: int, Rk: np.ndarray, c: float, mode: int, source_max: int = MAX_SOURCE_LEVEL,
         source_zsum: bool = True):
    """(l(k) int32[n], sum_{l<=l(k)} Z_l(k) float64[n], R'(k) uint64[n]).
    source_zsum=False leaves the source's sum as NaN (for graphs where
    Lemma 4 on the CPU is out of reach)."""
    n = g.n
    Rk = np.asarray(Rk, dtype=np.uint64)
    ell = np.zeros(n, dtype=np.int32)
    zsum = np.zeros(n)
    if mode == MODE_OFF:
        return ell, zsum, Rk.copy()
    sc = math.sqrt(c)
    budget = (2.0 * Rk.astype(np.float64)) / sc
    take = (Rk > 0) & (g.din.astype(np.float64) <= budget)
    ell[take] = 1
    has = take & (g.din > 0)
    zsum[has] = c / g.din[has].astype(np.float64)
    if Rk[u] > 0:
        e1, e2, e3 = edge_costs(g, u)
        work = (float(e1), float(e2), float(e2) + float(level3_path_cost(n)) * float(e3 - e2))
        lu = 0
        for l in range(1, source_max + 1):
            if work[l - 1] <= budget[u]:
                lu = l
        ell[u] = lu
        if not source_zsum:
            zsum[u] = np.nan
        else:
            zsum[u] = float(first_meeting(g, u, c, lu)[1:].sum()) if lu > 0 else 0.0
    if mode == MODE_REDUCED:
        cl = np.array([c_power(c, l) for l in range(source_max + 1)])
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
