"""Pins of the local deterministic exploitation oracle (Section 3.3,
Algorithm 3, Lemma 4)."""
import math

import numpy as np
import pytest

import workloads
from graphs import complete, cycle, random_graph, siblings, three_sources
from oracle import exactsim as ox
from oracle import lde
from oracle import simrank as sr
from oracle.graph import OracleGraph

C = 0.6

TINY = {
    "complete4": lambda: complete(4),
    "cycle5": lambda: cycle(5),
    "siblings": lambda: siblings(),
    "three_sources": lambda: three_sources(),
    "random8a": lambda: random_graph(8, 24, 1),
    "random8b": lambda: random_graph(8, 14, 2),
    "random10": lambda: random_graph(10, 35, 3),
}


@pytest.mark.parametrize("name", list(TINY))
def test_lemma4_equals_pair_enumeration(name):
    n, s, d = TINY[name]()
    g = OracleGraph(n, s, d)
    for k in range(n):
        z = lde.first_meeting(g, k, C, 5)
        b = lde.brute_first_meeting(g, k, C, 5)
        assert np.allclose(z, b, rtol=1e-12, atol=1e-15), (k, z, b)


def test_first_level_closed_form():
    n, s, d = random_graph(40, 200, 7)
    g = OracleGraph(n, s, d)
    for k in range(n):
        z = lde.first_meeting(g, k, C, 1)[1]
        want = C / g.din[k] if g.din[k] > 0 else 0.0
        assert z == pytest.approx(want, rel=1e-14, abs=0)


def test_first_meetings_add_up_to_one_minus_d():
    n, (s, d) = 60, workloads.chung_lu(60, 400, 5)
    g = OracleGraph(n, s, d)
    S = sr.power_method(g, C, 80)
    D = sr.exact_diagonal(g, S, C)
    L = 40
    for k in (0, 1, 7, 30, 59):
        z = lde.first_meeting(g, k, C, L)
        # meetings after step L need both walks alive at step L + 1
        assert abs((1.0 - z.sum()) - D[k]) <= C ** (L + 1) + 1e-12


def test_complete_graph_first_level():
    # K4: every node has the three others as in-neighbours; two walks meet
    # at step 1 with probability c/3
    n, s, d = complete(4)
    g = OracleGraph(n, s, d)
    assert lde.first_meeting(g, 0, C, 1)[1] == pytest.approx(C / 3, rel=1e-15)


def test_nonstop_zero_is_plain_algorithm_2():
    n, (s, d) = 300, workloads.chung_lu(300, 2500, 9)
    g = OracleGraph(n, s, d)
    R = np.random.default_rng(1).integers(0, 300, n).astype(np.uint64)
    a = ox.walk_counts(g, R, 17, C)
    b = ox.walk_counts(g, R, 17, C, nonstop=np.zeros(n, dtype=np.int32))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("l", [1, 2, 3])
def test_nonstop_pairs_meet_at_the_tail_probability(l):
    # the fraction of non-stop pairs that meet after step l estimates
    # c^-l sum_{t > l} Z_t(k)
    n, (s, d) = 80, workloads.chung_lu(80, 500, 4)
    g = OracleGraph(n, s, d)
    k = int(np.argmax(g.din))
    z = lde.first_meeting(g, k, C, 45)
    p = z[l + 1:].sum() / C ** l
    R = 400_000
    Rk = np.zeros(n, dtype=np.uint64)
    Rk[k] = R
    ns = np.full(n, l, dtype=np.int32)
    M = int(ox.walk_counts(g, Rk, 31 + l, C, nonstop=ns)[k])
    sigma = math.sqrt(p * (1 - p) / R)
    assert abs(M / R - p) <= 6 * sigma + C ** 45


def test_estimator_is_unbiased():
    n, (s, d) = 80, workloads.chung_lu(80, 500, 4)
    g = OracleGraph(n, s, d)
    S = sr.power_method(g, C, 80)
    D = sr.exact_diagonal(g, S, C)
    nodes = np.argsort(-g.din)[:6]
    Rk = np.zeros(n, dtype=np.uint64)
    Rk[nodes] = 200_000
    for l in (1, 2):
        ell = np.zeros(n, dtype=np.int32)
        ell[nodes] = l
        zsum = np.zeros(n)
        for k in nodes:
            zsum[k] = lde.first_meeting(g, int(k), C, l)[1:].sum()
        M = ox.walk_counts(g, Rk, 90 + l, C, nonstop=ell)
        Dh = lde.diag_estimate(Rk, M, ell, zsum, C, g.din)
        for k in nodes:
            tail = 1.0 - zsum[k] - D[k]          # = sum_{t > l} Z_t(k)
            p = tail / C ** l
            sigma = C ** l * math.sqrt(max(p * (1 - p), 1e-12) / 200_000)
            assert abs(Dh[k] - D[k]) <= 6 * sigma + 1e-12


def test_estimator_formula_and_shortcuts():
    din = np.array([0, 1, 2, 5, 3])
    Rk = np.array([0, 0, 10, 7, 4], dtype=np.uint64)
    M = np.array([0, 0, 3, 2, 1], dtype=np.uint64)
    ell = np.array([0, 0, 0, 1, 2], dtype=np.int32)
    zsum = np.array([0, 0, 0, C / 5, 0.25])
    D = lde.diag_estimate(Rk, M, ell, zsum, C, din)
    assert D[0] == 1.0 and D[1] == 1.0 - C
    assert D[2] == 7.0 / 10.0
    assert D[3] == (1.0 - C / 5) - C * (2.0 / 7.0)
    assert D[4] == (1.0 - 0.25) - (C * C) * (1.0 / 4.0)


def test_plan_rule():
    n, (s, d) = 500, workloads.chung_lu(500, 4000, 8)
    g = OracleGraph(n, s, d)
    u = int(np.argmax(g.din))
    L = ox.num_levels(C, 1e-4)
    _, pi = ox.forward_levels(g, u, C, L)
    R = ox.total_samples(n, C, 1e-4, 1e-3)
    Rk = ox.budget(pi, g.din, R)
    off_ell, _, off_R = lde.plan(g, u, Rk, C, lde.MODE_OFF)
    assert not off_ell.any() and np.array_equal(off_R, Rk)
    ell, zsum, R1 = lde.plan(g, u, Rk, C, lde.MODE_AS_PRINTED)
    assert np.array_equal(R1, Rk)
    others = np.arange(n) != u
    assert ell[others].max() <= 1 and ell[u] >= 1
    budget = 2.0 * Rk.astype(np.float64) / math.sqrt(C)
    one = others & (ell == 1)
    assert np.all(g.din[one] <= budget[one])
    assert np.all(g.din[others & (Rk > 0) & (ell == 0)] > budget[others & (Rk > 0) & (ell == 0)])
    assert np.all(zsum[one] == C / g.din[one].astype(np.float64))
    e = lde.edge_costs(g, u)
    work = (e[0], e[1], e[1] + lde.level3_path_cost(n) * (e[2] - e[1]))
    assert ell[u] == max(l for l in (0, 1, 2, 3) if l == 0 or work[l - 1] <= budget[u])
    _, _, R2 = lde.plan(g, u, Rk, C, lde.MODE_REDUCED)
    cl = np.array([1.0, C, C * C, C * C * C])
    assert np.array_equal(R2, np.ceil(Rk.astype(np.float64) * cl[ell]).astype(np.uint64))
    assert R2.sum() < Rk.sum()
