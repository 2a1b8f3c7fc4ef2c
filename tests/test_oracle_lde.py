"""Pins of the local deterministic exploitation oracle (Section 3.2,
Algorithm 3, Lemma 4)."""
import math

import numpy as np
import pytest

import workloads
from graphs import complete, cycle, diamond, fork, lde_rounds, random_graph, siblings, three_sources
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


GOLDEN_GRAPHS = {"complete4": lambda: complete(4), "diamond": diamond, "fork": fork,
                 "three_sources": three_sources}


@pytest.mark.parametrize("name", list(GOLDEN_GRAPHS))
def test_edge_counts_hand_counted(name):
    """Edges per round of Algorithm 3's loops against hand counts
    (tests/golden/lde_rounds.txt): the literal loops and the C counter."""
    k, want = lde_rounds()[name]
    n, s, d = GOLDEN_GRAPHS[name]()
    g = OracleGraph(n, s, d)
    ell, _, costs = lde.printed_exploitation(g, k, C, math.inf, cap=len(want))
    ended = want[-1] == 0
    assert costs == want
    assert ell == (len(want) - 1 if ended else len(want))
    l2, c2 = lde.printed_levels(g, [k], [math.inf], len(want), with_costs=True)
    assert l2[0] == ell
    assert list(c2[0][:len(want)]) == want


@pytest.mark.parametrize("T,want", [(1.0, 0), (2.0, 0), (2.5, 1), (6.0, 1), (6.25, 2), (10.0, 2), (10.5, 3),
                                    (15.0, 3), (15.5, 4), (27.0, 4), (27.5, 5)])
def test_level_is_the_round_where_the_budget_is_reached(T, want):
    """diamond, node 0: cumulative counts 2, 6, 10, 15, 27 (hand count); the
    exploitation stops in the round where E_k reaches T."""
    n, s, d = diamond()
    g = OracleGraph(n, s, d)
    assert lde.printed_exploitation(g, 0, C, T, cap=8)[0] == want
    assert lde.printed_levels(g, [0], [T], 8)[0] == want
    # a cap cuts the level and never raises it
    for cap in range(0, 6):
        assert lde.printed_levels(g, [0], [T], cap)[0] == min(want, cap)
        assert lde.printed_exploitation(g, 0, C, T, cap=cap)[0] == min(want, cap)


def test_exhausted_exploitation_is_exact():
    """fork: round 2 traverses nothing, so l(0) = 2 whatever the budget and
    the exact part is all of 1 - D(0,0) = c/2 (no walk survives step 2)."""
    n, s, d = fork()
    g = OracleGraph(n, s, d)
    for T in (7.0, 1e6, math.inf):
        ell, Z, _ = lde.printed_exploitation(g, 0, C, T, cap=10)
        assert ell == 2 and lde.printed_levels(g, [0], [T], 10)[0] == 2
        assert sum(Z) == pytest.approx(C / 2, rel=1e-15)
    S = sr.power_method(g, C, 80)
    assert 1.0 - sr.exact_diagonal(g, S, C)[0] == pytest.approx(C / 2, rel=1e-12)


@pytest.mark.parametrize("name", list(TINY))
def test_printed_rounds_give_lemma4_and_enumeration(name):
    """The Z_l the printed rounds evaluate (Lemma 4 on the tables they build)
    equal first meetings enumerated over pairs of walks."""
    n, s, d = TINY[name]()
    g = OracleGraph(n, s, d)
    for k in range(n):
        ell, Z, _ = lde.printed_exploitation(g, k, C, math.inf, cap=5)
        b = lde.brute_first_meeting(g, k, C, ell)
        assert np.allclose(Z[:ell + 1], b, rtol=1e-12, atol=1e-15), (k, Z, b)


def brute_round_costs(g, k, rounds):
    """Edges per round counted from the definition with plain Python sets:
    for each l' and each q' reached from v_k in exactly l - l' steps, the
    in-degrees of the nodes reached from q' in exactly l' steps."""
    def reach(v, j):
        cur = {v}
        for _ in range(j):
            cur = {int(q) for x in cur for q in g.in_neighbours(x)}
        return cur
    out = []
    for l in range(rounds):
        out.append(sum(int(g.din[x]) for lp in range(l + 1) for q2 in reach(k, l - lp) for x in reach(q2, lp)))
    return out


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_c_counter_matches_printed_loops_and_sets(seed):
    """On random graphs: rounds counted by the C counter, by the literal
    loops and by set arithmetic agree, and so do the levels for random
    budgets (including budgets met exactly at a round's end)."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(6, 25))
    _, s, d = random_graph(n, int(rng.integers(n, 4 * n)), seed)
    g = OracleGraph(n, s, d)
    nodes = np.arange(n, dtype=np.int32)
    _, costs = lde.printed_levels(g, nodes, np.full(n, math.inf), 4, with_costs=True)
    for k in range(n):
        brute = brute_round_costs(g, k, 4)
        ell, _, lit = lde.printed_exploitation(g, k, C, math.inf, cap=4)
        if 0 in brute:
            brute = brute[:brute.index(0) + 1]
        assert lit == brute, (k, lit, brute)
        assert list(costs[k][:len(brute)]) == brute
        cum = np.cumsum(brute)
        Ts = list(rng.uniform(0, cum[-1] * 1.2, 5)) + [float(x) for x in cum]
        for T in Ts:
            a = lde.printed_exploitation(g, k, C, T, cap=4)[0]
            b = lde.printed_levels(g, [k], [T], 4)[0]
            assert a == b, (k, T, a, b)


def test_plan_every_node_by_the_same_rule():
    """plan(): every sampled node (the query source is not special) gets
    min(l_printed, cap); Z by Lemma 4; R' per mode."""
    n, (s, d) = 400, workloads.chung_lu(400, 3000, 8)
    g = OracleGraph(n, s, d)
    u = int(np.argmax(g.din))
    L = ox.num_levels(C, 1e-4)
    _, pi = ox.forward_levels(g, u, C, L)
    Rk = ox.budget(pi, g.din, ox.total_samples(n, C, 1e-4, 1e-2))
    off_ell, _, off_R = lde.plan(g, Rk, C, lde.MODE_OFF)
    assert not off_ell.any() and np.array_equal(off_R, Rk)
    for cap in (1, 2, 3):
        ell, zsum, R1 = lde.plan(g, Rk, C, lde.MODE_AS_PRINTED, max_level=cap)
        assert np.array_equal(R1, Rk)
        act = np.flatnonzero(Rk > 0)
        assert np.all(ell[Rk == 0] == 0)
        T = lde.edge_budget(Rk, C)
        for k in act[:: max(1, len(act) // 40)]:
            want = lde.printed_exploitation(g, int(k), C, T[k], cap=cap)
            assert ell[k] == want[0]
            assert zsum[k] == pytest.approx(sum(want[1]), rel=1e-12, abs=1e-15)
        if cap >= 2:
            assert (ell >= 2).sum() > 0 and ell.max() == cap
        one = ell == 1
        assert np.all(zsum[one] == C / g.din[one].astype(np.float64))
    _, _, R2 = lde.plan(g, Rk, C, lde.MODE_REDUCED, max_level=3)
    cl = np.array([1.0, C, C * C, C * C * C])
    assert np.array_equal(R2, np.ceil(Rk.astype(np.float64) * cl[ell]).astype(np.uint64))
    assert R2.sum() < Rk.sum()
