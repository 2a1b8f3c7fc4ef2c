"""Oracle view of a directed graph (test infrastructure).

Notation of Section 2: I(v) / O(v) are the in- / out-neighbour sets,
d_in(v) = |I(v)|, and the (reverse) transition matrix has
P(i, j) = 1 / d_in(v_j) for v_i in I(v_j), else 0.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class OracleGraph:
    """Edge set (src -> dst) with the matrices the oracle needs.

    Duplicate edges are merged and self-loops kept only if asked: SimRank's
    definition (Eq. 1) sums over neighbour sets.
    """

    def __init__(self, n: int, src, dst, keep_self_loops: bool = False):
        src = np.asarray(src, dtype=np.int64)
        dst = np.asarray(dst, dtype=np.int64)
        if not keep_self_loops:
            keep = src != dst
            src, dst = src[keep], dst[keep]
        key = np.unique(src * n + dst)
        self.n = n
        self.src = (key // n).astype(np.int64)
        self.dst = (key % n).astype(np.int64)
        self.m = len(key)
        self.din = np.bincount(self.dst, minlength=n).astype(np.int64)
        self.dout = np.bincount(self.src, minlength=n).astype(np.int64)
        with np.errstate(divide="ignore"):
            self.inv_din = np.where(self.din > 0, 1.0 / np.maximum(self.din, 1), 0.0)
        # A[i, j] = 1 iff (v_i -> v_j) is an edge, i.e. v_j in O(v_i), v_i in I(v_j).
        self.A_int = sp.csr_matrix((np.ones(self.m, dtype=np.int64), (self.src, self.dst)), shape=(n, n))
        self.A = self.A_int.astype(np.float64)
        self.AT = sp.csr_matrix(self.A.T)
        # P = A diag(1/d_in)
        self.P = sp.csr_matrix(self.A @ sp.diags(self.inv_din))
        self.PT = sp.csr_matrix(self.P.T)
        # In-neighbour lists in ascending id order (the walk sampler's order).
        order = np.lexsort((self.src, self.dst))
        self.in_idx = self.src[order].astype(np.int32)
        self.in_off = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(self.din, out=self.in_off[1:])

    def in_neighbours(self, v: int) -> np.ndarray:
        return self.in_idx[self.in_off[v]:self.in_off[v + 1]]

    def dense_P(self) -> np.ndarray:
        return self.P.toarray()
