"""Pins of the oracle's sparse linearization (Section 3.2, Lemma 2).

Sparse linearization stores only the entries pi^l(k) > theta =
(1 - sqrt c)^2 eps_s of the l-hop PPR levels.  The pins: a directed cycle,
where the kept levels and s(u, u) have closed forms; Lemma 2's error bound
against the Power Method's exact diagonal; the effect of the removed entries
recomputed through the PPR-pairs form of Section 2 with plain dense matrix
powers; the pigeonhole count bound; and the boundary cases.
"""
import math

import numpy as np
import pytest

import workloads
from graphs import cycle, random_graph
from oracle import exactsim as ox
from oracle import simrank as sr
from oracle.graph import OracleGraph

C = 0.6


def test_threshold_value():
    # (1 - sqrt 0.6)^2 = 1.6 - 2 sqrt 0.6
    want = (1.6 - 2.0 * math.sqrt(0.6)) * 1e-6
    assert ox.sparse_threshold(C, 1e-6) == pytest.approx(want, rel=1e-12)
    assert ox.sparse_threshold(C, 0.0) == 0.0


def test_cycle_closed_form():
    # On a directed cycle longer than L + 1 every level holds one entry,
    # pi^l(u - l) = (1 - sqrt c) sqrt(c)^l, and with D = 1 - c everywhere
    # s(u, u) = (1 - c) sum_{l kept} c^l = 1 - c^(l* + 1), s(u, v) = 0.
    n = 40
    g = OracleGraph(*cycle(n))
    eps, eps_s = 1e-4, 0.05
    L = ox.num_levels(C, eps)
    assert L == 20
    sc = math.sqrt(C)
    theta = (1 - sc) ** 2 * eps_s
    kept_levels = [l for l in range(L + 1) if (1 - sc) * sc ** l > theta]
    lstar = max(kept_levels)
    assert lstar == 17 and kept_levels == list(range(18))  # the cut is 10% away from either side
    u = 7
    q = ox.query(g, u, C, eps, 1, sparse_eps=eps_s)
    assert int(q["Rk"].sum()) == 0  # d_in = 1 everywhere: exact diagonal
    nz = [(l, int(k)) for l in range(L + 1) for k in np.flatnonzero(q["kept"][l])]
    assert nz == [(l, (u - l) % n) for l in range(lstar + 1)]
    want = np.zeros(n)
    want[u] = 1 - C ** (lstar + 1)
    assert np.abs(q["s"] - want).max() < 1e-15
    # the dense query keeps all L + 1 levels
    dense = ox.query(g, u, C, eps, 1)
    assert dense["s"][u] == pytest.approx(1 - C ** (L + 1), abs=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_lemma2_error_bound(seed):
    # With the exact diagonal (values in [1 - c, 1]) the removed entries lower
    # every s(u, j) by at least 0 and at most eps_s.
    n, m = 300, 2400
    src, dst = workloads.chung_lu(n, m, 40 + seed)
    g = OracleGraph(n, src, dst)
    S = sr.power_method(g, C, 70)
    D = sr.exact_diagonal(g, S, C)
    eps = 1e-5
    for eps_s in (1e-2, 1e-3, 1e-4):
        for u in (0, 17, 123):
            dense = ox.query(g, u, C, eps, 1, d_override=D)
            sparse = ox.query(g, u, C, eps, 1, d_override=D, sparse_eps=eps_s)
            diff = dense["s"] - sparse["s"]
            assert diff.min() >= -1e-15
            assert diff.max() <= eps_s
            removed = (dense["levels"] > 0) & (sparse["kept"] == 0)
            assert removed.any()


def _dense_ppr_levels(g, i, c, L):
    """pi_i^l = (1 - sqrt c)(sqrt c P)^l e_i for l = 0..L as dense float64 matrix powers."""
    sc = math.sqrt(c)
    P = g.P.toarray() if hasattr(g.P, "toarray") else np.asarray(g.P)
    out = np.zeros((L + 1, g.n))
    M = np.eye(g.n)
    for l in range(L + 1):
        out[l] = (1 - sc) * M[:, i]
        M = (sc * P) @ M
    return out


def test_removed_mass_through_ppr_pairs():
    # s(u, j) = (1 - sqrt c)^-2 sum_l sum_k pi_u^l(k) pi_j^l(k) D(k) (Section 2),
    # so the sparse result must equal that sum over the kept (l, k) only.
    n, s, d = random_graph(60, 420, 5)
    g = OracleGraph(n, s, d)
    rng = np.random.default_rng(3)
    D = rng.uniform(1 - C, 1.0, g.n)
    eps, eps_s = 1e-4, 2e-2
    L = ox.num_levels(C, eps)
    sc = math.sqrt(C)
    theta = (1 - sc) ** 2 * eps_s
    u = int(np.argmax(g.din))
    pu = _dense_ppr_levels(g, u, C, L)
    keep = pu > theta
    sparse = ox.query(g, u, C, eps, 1, d_override=D, sparse_eps=eps_s)
    assert (keep == (sparse["kept"] > 0)).all()
    for j in range(g.n):
        pj = _dense_ppr_levels(g, j, C, L)
        want = float(np.sum(np.where(keep, pu * pj, 0.0) * D)) / (1 - sc) ** 2
        assert sparse["s"][j] == pytest.approx(want, abs=1e-13)


@pytest.mark.parametrize("seed", [0, 1])
def test_pigeonhole_count_bound(seed):
    # the levels' total mass is at most 1, so at most 1/theta entries exceed theta
    n, m = 3000, 30000
    src, dst = workloads.rmat(n, m, 90 + seed)
    g = OracleGraph(n, src, dst)
    eps = 1e-6
    L = ox.num_levels(C, eps)
    levels, _ = ox.forward_levels(g, 5, C, L)
    assert levels.sum() <= 1.0 + 1e-12
    for eps_s in (1e-2, 1e-3, 1e-4):
        theta = ox.sparse_threshold(C, eps_s)
        kept = int(np.count_nonzero(ox.sparsify_levels(levels, theta)))
        assert 0 < kept <= 1.0 / theta
        assert kept == int(np.count_nonzero(levels > theta))


def test_tiny_threshold_is_the_dense_query():
    src, dst = workloads.chung_lu(500, 4000, 9)
    g = OracleGraph(500, src, dst)
    dense = ox.query(g, 3, C, 1e-3, 7, r_scale=1e-4)
    sparse = ox.query(g, 3, C, 1e-3, 7, r_scale=1e-4, sparse_eps=1e-300)
    assert np.array_equal(dense["s"], sparse["s"])
    # the walk budget is the one of the full vectors in both
    assert np.array_equal(dense["Rk"], sparse["Rk"])


def test_entry_at_threshold_is_removed():
    levels = np.array([[0.0, 0.25, 0.5], [0.125, 0.0, 0.375]])
    out = ox.sparsify_levels(levels, 0.25)
    assert out.tolist() == [[0.0, 0.0, 0.5], [0.0, 0.0, 0.375]]
    assert levels[0, 1] == 0.25  # the input is not modified
