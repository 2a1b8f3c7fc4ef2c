"""Pins of the CPU oracle against facts fixed outside it.

Each test checks an oracle function against something other than itself:
numpy's Philox, exact rational or high-precision decimal arithmetic, closed
forms derived from Eq. 1, a direct linear solve of Eq. 1, brute-force
enumeration, or the statistical law of the estimator.
"""
import math
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import workloads
from graphs import complete, cycle, golden, random_graph, siblings, three_sources
from oracle import exactsim as ox
from oracle import simrank as sr
from oracle.graph import OracleGraph

C = 0.6


def G(spec, **kw):
    n, s, d = spec
    return OracleGraph(n, s, d, **kw)


# ---------------------------------------------------------------- random numbers

@pytest.mark.parametrize("key,ctr", [
    ((0, 0), (0, 0, 0, 0)),
    ((1, 2), (3, 4, 5, 6)),
    ((2**64 - 1, 12345), (2**64 - 1, 2**63, 7, 0)),
    ((0xDEADBEEF, 0xCAFEF00D), (123456789, 987654321, 2**40, 2**62)),
])
def test_philox_matches_numpy(key, ctr):
    # numpy's Philox bit generator is Philox4x64-10; it increments its counter
    # before producing a block, so starting it at ctr - 1 yields block(ctr).
    as_int = sum(int(w) << (64 * i) for i, w in enumerate(ctr))  # 256-bit counter, word 0 lowest
    as_int = (as_int - 1) % 2**256
    pre = [(as_int >> (64 * i)) & (2**64 - 1) for i in range(4)]
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(pre, dtype=np.uint64))
    ref = bg.random_raw(4)
    got = ox.philox4x64_10(np.array(ctr, dtype=np.uint64), np.array(key, dtype=np.uint64))
    assert np.array_equal(ref, got)


def test_philox_numpy_counter_convention():
    bg = np.random.Philox(key=np.array([5, 6], dtype=np.uint64), counter=np.array([9, 0, 0, 0], dtype=np.uint64))
    bg.random_raw(4)
    assert int(bg.state["state"]["counter"][0]) == 10


def test_mulhi_exact_identity():
    rng = np.random.default_rng(1)
    for _ in range(2000):
        w = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        d = int(rng.integers(1, 2**31))
        assert ox.mulhi64(w, d) == (w * d) >> 64


def test_mulhi_uniform_on_stratified_grid():
    # words spread evenly over [0, 2^64): every index in [0, d) gets the same
    # count up to one
    d = 7
    N = 7 * 1000
    counts = np.zeros(d, dtype=int)
    for t in range(N):
        w = (t * (2**64 // N)) + (2**64 // N) // 2
        counts[ox.mulhi64(w, d)] += 1
    assert counts.max() - counts.min() <= 1


@pytest.mark.parametrize("c", [0.6, 0.8, 0.3])
def test_lifetime_thresholds_match_powers_of_c(c):
    thr = ox.c_lifetime_thresholds(c)
    assert np.array_equal(thr, ox.lifetime_thresholds(c))
    cf = Fraction(c)
    for t in range(1, len(thr)):
        exact = cf ** t * 2**64
        # floor of a value within t ulps of exact
        assert abs(Fraction(int(thr[t])) - exact) <= exact * Fraction(t + 2, 2**52) + 1
    # beyond the table, c^t 2^64 < 1
    assert cf ** len(thr) * 2**64 < 1
    assert all(thr[i] >= thr[i + 1] for i in range(1, len(thr) - 1))


# ---------------------------------------------------------------- host constants

@pytest.mark.parametrize("eps", [1e-1, 3e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7])
def test_num_levels_is_ceil_log(eps):
    L = ox.num_levels(C, eps)
    x = math.log(2.0 / eps) / math.log(1.0 / C)
    assert abs(x - round(x)) > 1e-9  # not on an integer boundary
    assert L == math.ceil(x)
    assert C ** L <= eps / 2 < C ** (L - 1)


def test_levels_at_paper_settings():
    # c = 0.6: eps 1e-4 -> L = 20, eps 1e-6 -> L = 29
    assert ox.num_levels(0.6, 1e-4) == 20
    assert ox.num_levels(0.6, 1e-6) == 29


@pytest.mark.parametrize("n,eps", [(2000, 1e-4), (2**20, 1e-6), (42_000_000, 1e-6), (5, 0.5)])
def test_total_samples_high_precision(n, eps):
    getcontext().prec = 50
    c = Decimal(C)
    om = 1 - c.sqrt()
    ref = 6 * Decimal(n).ln() / (om ** 4 * Decimal(eps) ** 2)
    got = Decimal(ox.total_samples(n, C, eps))
    assert abs(got - ref) / ref < Decimal("1e-14")


# ---------------------------------------------------------------- ground truth

@pytest.mark.parametrize("n", [3, 4, 5])
def test_power_method_complete_graph(n):
    g = G(complete(n))
    S = sr.power_method(g, C, 80)
    want = golden(f"K{n}")
    off = S[~np.eye(n, dtype=bool)]
    assert np.allclose(off, want, atol=1e-14, rtol=0)
    assert np.allclose(np.diag(S), 1.0)


def test_power_method_siblings_cycle_sources():
    S = sr.power_method(G(siblings()), C, 80)
    assert abs(S[1, 2] - golden("siblings")) < 1e-15
    assert S[0, 1] == 0.0 and S[0, 2] == 0.0  # v_0 has no in-neighbour
    S = sr.power_method(G(cycle(7)), C, 80)
    assert np.abs(S - np.eye(7)).max() == golden("cycle_offdiag")


@pytest.mark.parametrize("seed", range(6))
def test_power_method_matches_direct_solve(seed):
    g = G(random_graph(6, 14, seed))
    S = sr.power_method(g, C, 90)
    S2 = sr.pair_solve(g, C)
    assert np.abs(S - S2).max() < 1e-13
    assert np.allclose(S, S.T, atol=1e-15)


def test_power_method_truncation_bound():
    g = G(random_graph(7, 20, 9))
    exact = sr.pair_solve(g, C)
    for T in (3, 6, 10):
        err = np.abs(sr.power_method(g, C, T) - exact).max()
        assert err <= C ** (T + 1) + 1e-15


def test_exact_diagonal_special_cases():
    g = G(three_sources())
    S = sr.power_method(g, C, 80)
    D = sr.exact_diagonal(g, S, C)
    assert abs(D[0] - golden("D_three_sources")) < 1e-15
    assert D[1] == golden("D_din0")
    g = G(cycle(5))
    D = sr.exact_diagonal(g, sr.power_method(g, C, 80), C)
    assert np.allclose(D, golden("D_din1"), atol=1e-15)


def test_exact_diagonal_range_and_meeting_probability():
    g = G(random_graph(6, 14, 3))
    S = sr.pair_solve(g, C)
    D = sr.exact_diagonal(g, S, C)
    assert np.all(D >= 1 - C - 1e-15) and np.all(D <= 1 + 1e-15)
    # S = sum_l c^l (P^l)^T D P^l summed to convergence reproduces S
    P = g.dense_P()
    acc = np.zeros_like(S)
    Pl = np.eye(6)
    for l in range(120):
        acc += C ** l * Pl.T @ np.diag(D) @ Pl
        Pl = P @ Pl
    assert np.abs(acc - S).max() < 1e-13


def test_meeting_probability_by_path_enumeration():
    # Pr[two sqrt(c)-walks from v_k meet] by summing over every pair of paths
    # up to length 12 (first meeting only); compare with 1 - D(k, k)
    g = G(random_graph(5, 11, 4))
    D = sr.exact_diagonal(g, sr.pair_solve(g, C), C)
    for k in range(5):
        prob = 0.0
        frontier = {(k, k): 1.0}  # joint positions of walks that have not met
        for t in range(1, 40):
            nxt = {}
            for (x, y), p in frontier.items():
                Ix, Iy = g.in_neighbours(x), g.in_neighbours(y)
                if len(Ix) == 0 or len(Iy) == 0:
                    continue
                q = p * C / (len(Ix) * len(Iy))
                for a in Ix:
                    for b in Iy:
                        if a == b:
                            prob += q
                        else:
                            nxt[(int(a), int(b))] = nxt.get((int(a), int(b)), 0.0) + q
            frontier = nxt
        assert abs((1 - prob) - D[k]) < 1e-8


def test_linearization_with_exact_D_matches_power_method():
    src, dst = workloads.chung_lu(300, 2400, 5)
    g = OracleGraph(300, src, dst)
    S = sr.power_method(g, C, 70)
    D = sr.exact_diagonal(g, S, C)
    for L in (5, 10, 20):
        for u in (0, 7, 123):
            s = sr.linearized_column(g, u, C, L, D)
            assert np.abs(s - S[:, u]).max() <= C ** (L + 1) + 1e-12


def test_ppr_pair_form_equals_linearization():
    g = G(random_graph(30, 120, 8))
    D = np.linspace(0.45, 0.95, 30)
    s = sr.linearized_column(g, 3, C, 15, D)
    for j in (0, 3, 17, 29):
        assert abs(sr.ppr_pairs_form(g, 3, j, C, 15, D) - s[j]) < 1e-14


# ---------------------------------------------------------------- forward pass

def test_forward_close_to_plain_float64():
    src, dst = workloads.rmat(4096, 40000, 3)
    g = OracleGraph(4096, src, dst)
    L = 12
    levels, pi = ox.forward_levels(g, 5, C, L)
    sc = math.sqrt(C)
    ref = np.zeros(4096)
    ref[5] = 1 - sc
    bound = (g.dout.astype(float) + 1) * 2.0 ** -62
    for l in range(1, L + 1):
        ref = sc * (g.P @ ref)
        # rounding of the terms and of the previous level compound over levels
        assert np.all(np.abs(levels[l] - ref) <= l * bound + 1e-300)
    assert np.array_equal(pi, np.sum(levels[: L + 1], axis=0)) or np.abs(pi - levels.sum(0)).max() < 1e-16


def test_forward_cycle_closed_form():
    n = 40
    g = G(cycle(n))
    L = 25
    levels, _ = ox.forward_levels(g, 10, C, L)
    sc = math.sqrt(C)
    for l in range(L + 1):
        want = np.zeros(n)
        want[(10 - l) % n] = (1 - sc) * sc ** l
        # float64 rounding of both sides (relative) plus one 2^-62 quantum per level
        tol = (1 - sc) * sc ** l * (l + 2) * 2.0 ** -52 + (l + 1) * 2.0 ** -62
        assert np.abs(levels[l] - want).max() <= tol


def test_forward_mass_identity():
    # every node has an in-neighbour: sum_k pi^l(k) = (1 - sqrt c) sqrt(c)^l
    n, s, d = cycle(200)
    rng = np.random.default_rng(2)
    s = np.concatenate([s, rng.integers(0, n, 600)])
    d = np.concatenate([d, rng.integers(0, n, 600)])
    g = OracleGraph(n, s, d)
    assert g.din.min() >= 1
    levels, _ = ox.forward_levels(g, 3, C, 20)
    sc = math.sqrt(C)
    for l in range(21):
        assert abs(levels[l].sum() - (1 - sc) * sc ** l) < n * 2.0 ** -60


# ---------------------------------------------------------------- budget, walks

def test_budget_pi2_and_small_din():
    pi = np.array([0.0, 0.5, 1e-9, 0.25, 0.125])  # squares exact in binary
    din = np.array([3, 3, 3, 1, 0])
    Rk = ox.budget(pi, din, 1000.0, exact_small_din=True)
    assert Rk.tolist() == [0, 250, 1, 0, 0]
    Rk = ox.budget(pi, din, 1000.0, exact_small_din=False)
    assert Rk.tolist() == [0, 250, 1, 63, 16]
    assert ox.budget_pi(pi, din, 1000.0, exact_small_din=False).tolist() == [0, 500, 1, 250, 125]


def _sigma_ok(M, R, p, z=6.0):
    sd = math.sqrt(R * p * (1 - p)) if 0 < p < 1 else 0.0
    return abs(M - R * p) <= z * sd + 1e-9


def test_walks_meet_probability_three_sources():
    g = G(three_sources())
    R = 200_000
    Rk = np.array([R, 0, 0, 0], dtype=np.uint64)
    M = ox.walk_counts(g, Rk, seed=7, c=C)
    assert _sigma_ok(int(M[0]), R, C / 3)


def test_walks_cycle_meet_at_step_one():
    g = G(cycle(5))
    R = 100_000
    Rk = np.full(5, R, dtype=np.uint64)
    M = ox.walk_counts(g, Rk, seed=3, c=C)
    for k in range(5):
        assert _sigma_ok(int(M[k]), R, C)


def test_walks_match_exact_diagonal():
    g = G(random_graph(7, 22, 11))
    D = sr.exact_diagonal(g, sr.pair_solve(g, C), C)
    R = 300_000
    Rk = np.where(g.din > 0, R, 0).astype(np.uint64)
    M = ox.walk_counts(g, Rk, seed=5, c=C)
    for k in range(7):
        if g.din[k] > 0:
            assert _sigma_ok(int(M[k]), R, 1 - D[k]), (k, int(M[k]), R * (1 - D[k]))


def test_walks_split_ranges_add_up():
    src, dst = workloads.chung_lu(500, 4000, 9)
    g = OracleGraph(500, src, dst)
    rng = np.random.default_rng(0)
    Rk = rng.integers(0, 3000, 500).astype(np.uint64)
    mid = (Rk // 3).astype(np.uint64)
    full = ox.walk_counts(g, Rk, 21, C)
    a = ox.walk_counts(g, mid, 21, C)
    b = ox.walk_counts(g, Rk, 21, C, r_begin=mid)
    assert np.array_equal(full, a + b)
    assert np.array_equal(full, ox.walk_counts(g, Rk, 21, C, threads=1))


def test_walk_pair_is_pure_function_of_seed_node_sample():
    src, dst = workloads.chung_lu(200, 1500, 4)
    g = OracleGraph(200, src, dst)
    vals = [ox.walk_pair(g, 99, C, 0, r) for r in range(200)]
    assert vals == [ox.walk_pair(g, 99, C, 0, r) for r in range(200)]
    assert 0 < sum(vals) < 200


def test_diag_estimate_rules():
    Rk = np.array([10, 0, 0, 4], dtype=np.uint64)
    M = np.array([3, 0, 0, 4], dtype=np.uint64)
    din = np.array([5, 0, 1, 2])
    D = ox.diag_estimate(Rk, M, din, C)
    assert D.tolist() == [0.7, 1.0, 1.0 - C, 0.0]


# ---------------------------------------------------------------- whole query

def test_query_exact_D_matches_power_method():
    src, dst = workloads.chung_lu(400, 3500, 2)
    g = OracleGraph(400, src, dst)
    S = sr.power_method(g, C, 70)
    D = sr.exact_diagonal(g, S, C)
    for eps in (1e-2, 1e-4):
        L = ox.num_levels(C, eps)
        q = ox.query(g, 0, C, eps, 1, d_override=D)
        assert np.abs(q["s"] - S[:, 0]).max() <= C ** (L + 1) + 1e-12


def test_query_cycle_no_randomness():
    g = G(cycle(6))
    eps = 1e-3
    L = ox.num_levels(C, eps)
    q = ox.query(g, 2, C, eps, 1)
    assert int(q["Rk"].sum()) == 0  # d_in = 1 everywhere: exact D, no samples
    want = np.zeros(6)
    want[2] = 1 - C ** (L + 1)
    assert np.abs(q["s"] - want).max() < 1e-15


def test_query_source_without_in_neighbours():
    g = G(three_sources())
    q = ox.query(g, 2, C, 1e-3, 1)
    want = np.zeros(4)
    want[2] = 1.0
    assert np.abs(q["s"] - want).max() < 1e-15


@pytest.mark.parametrize("u", [0, 5, 77])
def test_query_error_within_eps(u):
    src, dst = workloads.chung_lu(300, 2400, 5)
    g = OracleGraph(300, src, dst)
    S = sr.power_method(g, C, 70)
    eps = 1e-2
    q = ox.query(g, u, C, eps, seed=17)
    assert sr.max_error(q["s"], S[:, u]) <= eps
    assert abs(q["s"][u] - 1.0) <= eps


def test_query_symmetry():
    src, dst = workloads.chung_lu(300, 2400, 5)
    g = OracleGraph(300, src, dst)
    eps = 1e-2
    a = ox.query(g, 5, C, eps, seed=3)["s"]
    b = ox.query(g, 9, C, eps, seed=4)["s"]
    assert abs(a[9] - b[5]) <= 2 * eps


def test_topk_brute_force():
    rng = np.random.default_rng(3)
    s = np.round(rng.random(500), 2)  # many ties
    idx, val = ox.topk(s, 7, 40)
    cand = sorted([(-s[j], j) for j in range(500) if j != 7])[:40]
    assert idx.tolist() == [j for _, j in cand]
    assert np.array_equal(val, s[idx])


def test_precision_at_k():
    s = np.array([1.0, 0.5, 0.4, 0.3, 0.2])
    t = np.array([1.0, 0.5, 0.3, 0.4, 0.2])
    assert sr.precision_at_k(s, t, 0, 2) == 0.5
    assert sr.precision_at_k(s, t, 0, 3) == 1.0
