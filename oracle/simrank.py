"""Exact SimRank ground truth in float64 (test infrastructure).

Each function follows a plain definition from the paper:

* ``power_method``      -- S_{t+1} = (c P^T S_t P) v I, S_0 = I (Section 2.1,
                           "Other Related Work"; the classic all-pairs method
                           the paper uses as ground truth on small graphs,
                           Section 4).  After T iterations the error is at most
                           c^(T+1) (Introduction: Power Method error c^L).
* ``pair_solve``        -- Eq. 1 of the Introduction written as a linear system
                           over ordered pairs (a, b), a != b, solved directly.
                           Exact up to rounding; used only on tiny graphs to pin
                           ``power_method`` independently.
* ``exact_diagonal``    -- D of the linearization S = sum_l c^l (P^l)^T D P^l
                           (Section 2, "Linearization and ParSim"): from
                           S = c P^T S P + D, D(k,k) = 1 - c (P^T S P)(k,k);
                           equivalently 1 - Pr[two sqrt(c)-walks from v_k meet]
                           (Section 3.2, local deterministic exploitation).
* ``linearized_column`` -- S e_i = 1/(1-sqrt c) sum_{l=0}^{L} (sqrt c P^T)^l D pi_i^l
                           with pi_i^l = (1-sqrt c)(sqrt c P)^l e_i (Section 3.1,
                           the rewrite of the single-source linearization), in
                           plain float64 with a given D.
"""
from __future__ import annotations

import math

import numpy as np

from .graph import OracleGraph


def power_method(g: OracleGraph, c: float, iters: int = 60) -> np.ndarray:
    """All-pairs SimRank matrix by the Power Method, dense float64."""
    n = g.n
    S = np.eye(n)
    PT = g.PT
    for _ in range(iters):
        X = PT @ S                # P^T S          (n x n dense)
        S = c * (PT @ X.T).T      # (P^T (P^T S)^T)^T = P^T S P
        np.fill_diagonal(S, 1.0)  # v I: diagonal of c P^T S P is <= c < 1
    return S


def pair_solve(g: OracleGraph, c: float) -> np.ndarray:
    """Solve Eq. 1 exactly as a linear system (tiny graphs only)."""
    n = g.n
    pairs = [(a, b) for a in range(n) for b in range(n) if a != b]
    index = {p: t for t, p in enumerate(pairs)}
    N = len(pairs)
    M = np.eye(N)
    rhs = np.zeros(N)
    for (a, b), row in index.items():
        Ia, Ib = g.in_neighbours(a), g.in_neighbours(b)
        if len(Ia) == 0 or len(Ib) == 0:
            continue  # empty sum: S(a, b) = 0
        w = c / (len(Ia) * len(Ib))
        for x in Ia:
            for y in Ib:
                if x == y:
                    rhs[row] += w          # S(x, x) = 1
                else:
                    M[row, index[(int(x), int(y))]] -= w
    sol = np.linalg.solve(M, rhs)
    S = np.eye(n)
    for (a, b), row in index.items():
        S[a, b] = sol[row]
    return S


def exact_diagonal(g: OracleGraph, S: np.ndarray, c: float) -> np.ndarray:
    """D(k,k) = 1 - c (P^T S P)(k,k); 1 for nodes without in-neighbours."""
    D = np.ones(g.n)
    for k in range(g.n):
        Ik = g.in_neighbours(k)
        d = len(Ik)
        if d == 0:
            continue
        D[k] = 1.0 - c * S[np.ix_(Ik, Ik)].sum() / (d * d)
    return D


def num_levels_ceil_log(c: float, eps: float) -> int:
    """L = ceil(log_{1/c}(2/eps)) of Algorithm 1 (float formula)."""
    return int(math.ceil(math.log(2.0 / eps) / math.log(1.0 / c)))


def linearized_column(g: OracleGraph, i: int, c: float, L: int, D: np.ndarray) -> np.ndarray:
    """Truncated linearization with diagonal D, plain float64 (no fixed point)."""
    sc = math.sqrt(c)
    pis = []
    pi = np.zeros(g.n)
    pi[i] = 1.0 - sc
    pis.append(pi)
    for _ in range(L):
        pi = sc * (g.P @ pi)
        pis.append(pi)
    s = D * pis[L] / (1.0 - sc)
    for l in range(1, L + 1):
        s = sc * (g.PT @ s) + D * pis[L - l] / (1.0 - sc)
    return s


def ppr_pairs_form(g: OracleGraph, i: int, j: int, c: float, L: int, D: np.ndarray) -> float:
    """S(i,j) = (1-sqrt c)^-2 sum_l sum_k pi_i^l(k) pi_j^l(k) D(k,k)
    (Section 2, PRSim paragraph; used in the proof of Theorem 1)."""
    sc = math.sqrt(c)
    pi_i = np.zeros(g.n)
    pi_i[i] = 1.0 - sc
    pi_j = np.zeros(g.n)
    pi_j[j] = 1.0 - sc
    tot = 0.0
    for _ in range(L + 1):
        tot += float(np.sum(pi_i * pi_j * D))
        pi_i = sc * (g.P @ pi_i)
        pi_j = sc * (g.P @ pi_j)
    return tot / (1.0 - sc) ** 2


def max_error(s: np.ndarray, truth: np.ndarray) -> float:
    """MaxError of Section 4: max_j |s(j) - S(i, j)|."""
    return float(np.max(np.abs(np.asarray(s) - np.asarray(truth))))


def precision_at_k(s: np.ndarray, truth: np.ndarray, i: int, k: int) -> float:
    """Precision@k of Section 4 (source excluded, ties to the smaller id)."""
    def top(v):
        idx = np.arange(len(v))
        keep = idx != i
        order = np.lexsort((idx[keep], -np.asarray(v)[keep]))
        return set(idx[keep][order[:k]].tolist())
    return len(top(s) & top(truth)) / float(k)
