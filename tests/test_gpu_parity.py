"""GPU parity: every step of the HIP path against the CPU oracle.

pi^l, R(k), M(k) and D^ must agree bit for bit; s within 1e-9 max-abs
(float64, summation order free); top-k exactly.  Inputs come from the seeded
generators only.
"""
import sys

import numpy as np
import pytest
import torch

import workloads
from graphs import complete, cycle, hub_graph, random_graph, three_sources
from oracle import exactsim as ox
from oracle import simrank as sr
from oracle.graph import OracleGraph

pytestmark = pytest.mark.gpu

C = 0.6
S_TOL = 1e-9


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def es():
    from paper_2004_03493_amd import binding
    return binding


@pytest.fixture(scope="module")
def ctx(es):
    c = es.Context(0)
    yield c
    c.close()


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype).cuda()


def u64(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.uint64)).cuda()


def host(t):
    return t.cpu().numpy()


GRAPHS = {
    "chung_lu_2k": lambda: (2000,) + workloads.chung_lu(2000, 20000, 11),
    "rmat_32k": lambda: (1 << 15,) + workloads.rmat(1 << 15, 500_000, 5),
    "hubs": lambda: hub_graph(30000, 20000, 20000, 60000, 3),
    "cycle": lambda: cycle(1000),
    "complete5": lambda: complete(5),
    "random_small": lambda: random_graph(50, 200, 1),
    "three_sources": lambda: three_sources(),
}


def build_pair(es, ctx, name):
    n, src, dst = GRAPHS[name]()
    say(f"[graph {name}] n={n} m={len(src)}")
    return es.Graph(ctx, n, src, dst), OracleGraph(n, src, dst)


@pytest.mark.parametrize("name", list(GRAPHS))
def test_forward_levels_bitwise(es, ctx, name):
    g, og = build_pair(es, ctx, name)
    assert g.m == og.m
    for u in sorted({0, og.n // 2, og.n - 1, int(np.argmax(og.din))}):
        for eps in (1e-4, 1e-6):
            L = ox.num_levels(C, eps)
            say(f"  forward u={u} L={L}")
            lv = torch.empty((L + 1) * g.n, dtype=torch.float64, device="cuda")
            pi = torch.empty(g.n, dtype=torch.float64, device="cuda")
            es.es_forward(ctx, g, u, C, L, lv, pi)
            ref_lv, ref_pi = ox.forward_levels(og, u, C, L)
            got = host(lv).reshape(L + 1, g.n)
            assert np.array_equal(got.view(np.uint64), ref_lv.view(np.uint64))
            assert np.array_equal(host(pi).view(np.uint64), ref_pi.view(np.uint64))


@pytest.mark.parametrize("name", ["chung_lu_2k", "rmat_32k", "hubs", "random_small"])
def test_budget_walks_diag_bitwise(es, ctx, name):
    g, og = build_pair(es, ctx, name)
    u = int(np.argmax(og.din))
    eps = 1e-4
    L = ox.num_levels(C, eps)
    target_pairs = 3e6
    for alloc, small in ((es.ES_ALLOC_PI2, True), (es.ES_ALLOC_PI2, False), (es.ES_ALLOC_PI, True)):
        ref_lv, ref_pi = ox.forward_levels(og, u, C, L)
        R0 = ox.total_samples(og.n, C, eps)
        raw = (ref_pi * ref_pi).sum() if alloc == es.ES_ALLOC_PI2 else ref_pi.sum()
        R = R0 * min(1.0, target_pairs / (R0 * raw + 1))
        budget = ox.budget if alloc == es.ES_ALLOC_PI2 else ox.budget_pi
        ref_R = budget(ref_pi, og.din, R, small)
        say(f"  budget alloc={alloc} small={small} R={R:.3g} pairs={int(ref_R.sum())}")
        lv = torch.empty((L + 1) * g.n, dtype=torch.float64, device="cuda")
        pi = torch.empty(g.n, dtype=torch.float64, device="cuda")
        es.es_forward(ctx, g, u, C, L, lv, pi)
        Rk = torch.empty(g.n, dtype=torch.uint64, device="cuda")
        tot = es.es_budget(ctx, g, pi, R, alloc, small, Rk, want_total=True)
        assert np.array_equal(host(Rk), ref_R)
        assert tot == int(ref_R.sum())
        say("  walks")
        M = torch.empty(g.n, dtype=torch.uint64, device="cuda")
        es.es_walk_pairs(ctx, g, None, Rk, 77, C, M)
        ref_M = ox.walk_counts(og, ref_R, 77, C)
        assert np.array_equal(host(M), ref_M)
        D = torch.empty(g.n, dtype=torch.float64, device="cuda")
        es.es_diag(ctx, g, Rk, M, C, small, D)
        ref_D = ox.diag_estimate(ref_R, ref_M, og.din, C, small)
        assert np.array_equal(host(D).view(np.uint64), ref_D.view(np.uint64))


@pytest.mark.parametrize("c", [0.002, 0.05])
def test_walks_small_decay(es, ctx, c):
    """A decay whose lifetime table ends within the walk kernel's unrolled
    thresholds (c^t 2^64 < 1 from t = 7 on at c = 0.002): meeting counts and
    D^ still equal the oracle's bit for bit."""
    g, og = build_pair(es, ctx, "rmat_32k")
    thr = ox.lifetime_thresholds(c)
    say(f"  c={c} lifetime table ends at t={len(thr) - 1}")
    rng = np.random.default_rng(9)
    R = rng.integers(0, 20_000, og.n).astype(np.uint64)
    R[og.din <= 1] = 0
    R[int(np.argmax(og.din))] = 2_000_000
    # a larger decay first leaves its thresholds in the context's table
    M0 = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    es.es_walk_pairs(ctx, g, None, u64(R), 3, 0.9, M0)
    M = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    es.es_walk_pairs(ctx, g, None, u64(R), 3, c, M)
    ref_M = ox.walk_counts(og, R, 3, c)
    assert ref_M.sum() > 0
    assert np.array_equal(host(M), ref_M)
    D = torch.empty(g.n, dtype=torch.float64, device="cuda")
    es.es_diag(ctx, g, u64(R), M, c, 1, D)
    ref_D = ox.diag_estimate(R, ref_M, og.din, c, True)
    assert np.array_equal(host(D).view(np.uint64), ref_D.view(np.uint64))


def test_walk_ranges_split_and_seed(es, ctx):
    g, og = build_pair(es, ctx, "rmat_32k")
    rng = np.random.default_rng(4)
    hi = rng.integers(0, 400, og.n).astype(np.uint64)
    hi[rng.random(og.n) < 0.5] = 0
    hi[int(np.argmax(og.din))] = 300_000
    lo = (hi // 3).astype(np.uint64)
    say(f"  ranges pairs={int(hi.sum())}")
    M_full = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    M_a = torch.empty_like(M_full)
    M_b = torch.empty_like(M_full)
    es.es_walk_pairs(ctx, g, None, u64(hi), 5, C, M_full)
    es.es_walk_pairs(ctx, g, None, u64(lo), 5, C, M_a)
    es.es_walk_pairs(ctx, g, u64(lo), u64(hi), 5, C, M_b)
    assert np.array_equal(host(M_full), host(M_a) + host(M_b))
    assert np.array_equal(host(M_b), ox.walk_counts(og, hi, 5, C, r_begin=lo))
    # repeated call is identical; another seed is not
    M_again = torch.empty_like(M_full)
    es.es_walk_pairs(ctx, g, None, u64(hi), 5, C, M_again)
    assert torch.equal(M_again, M_full)
    es.es_walk_pairs(ctx, g, None, u64(hi), 6, C, M_again)
    assert not torch.equal(M_again, M_full)


@pytest.mark.parametrize("c", [0.6, 0.8])
def test_walks_other_decay(es, ctx, c):
    g, og = build_pair(es, ctx, "chung_lu_2k")
    rng = np.random.default_rng(1)
    R = rng.integers(0, 2000, og.n).astype(np.uint64)
    M = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    es.es_walk_pairs(ctx, g, None, u64(R), 123, c, M)
    assert np.array_equal(host(M), ox.walk_counts(og, R, 123, c))


@pytest.mark.parametrize("name", ["chung_lu_2k", "rmat_32k", "hubs", "cycle"])
def test_backward_given_diagonal(es, ctx, name):
    g, og = build_pair(es, ctx, name)
    u = int(np.argmax(og.din))
    L = ox.num_levels(C, 1e-6)
    D = np.random.default_rng(2).uniform(1 - C, 1.0, og.n)
    ref_lv, _ = ox.forward_levels(og, u, C, L)
    lv = torch.empty((L + 1) * g.n, dtype=torch.float64, device="cuda")
    pi = torch.empty(g.n, dtype=torch.float64, device="cuda")
    es.es_forward(ctx, g, u, C, L, lv, pi)
    s = torch.empty(g.n, dtype=torch.float64, device="cuda")
    es.es_backward(ctx, g, lv, L, dev(D, torch.float64), C, s)
    ref = ox.back_accumulate(og, ref_lv, D, C)
    assert np.abs(host(s) - ref).max() <= 1e-12


@pytest.mark.parametrize("name,u,r_scale", [("chung_lu_2k", 0, 1e-3), ("rmat_32k", None, 1e-7),
                                            ("hubs", 1, 1e-6), ("three_sources", 2, 1.0),
                                            ("cycle", 5, 1.0), ("complete5", 0, 1e-2)])
def test_single_source_matches_oracle(es, ctx, name, u, r_scale):
    g, og = build_pair(es, ctx, name)
    if u is None:
        u = int(np.argmax(og.din))
    eps = 1e-4
    say(f"  query u={u} r_scale={r_scale}")
    s = torch.empty(g.n, dtype=torch.float64, device="cuda")
    st = es.es_single_source(ctx, g, u, es.make_opts(C, eps, 9, r_scale), s)
    ref = ox.query(og, u, C, eps, 9, r_scale)
    assert st.L == ref["L"] and st.R == ref["R"]
    assert st.pairs == int(ref["Rk"].sum())
    assert st.meets == int(ref["M"].sum())
    assert np.abs(host(s) - ref["s"]).max() <= S_TOL


def test_single_source_exact_D_vs_power_method(es, ctx):
    g, og = build_pair(es, ctx, "chung_lu_2k")
    say("  power method")
    S = sr.power_method(og, C, 60)
    D = sr.exact_diagonal(og, S, C)
    eps = 1e-6
    L = ox.num_levels(C, eps)
    Dt = dev(D, torch.float64)
    s = torch.empty(g.n, dtype=torch.float64, device="cuda")
    for u in (0, 17, 1999):
        es.es_single_source(ctx, g, u, es.make_opts(C, eps, 1, 1.0, d_override=Dt), s)
        assert np.abs(host(s) - S[:, u]).max() <= C ** (L + 1) + 1e-12


def test_single_source_accuracy_at_paper_budget_share(es, ctx):
    # 10% of the paper's sample budget still meets eps on the 2,000-node graph
    g, og = build_pair(es, ctx, "chung_lu_2k")
    S = sr.power_method(og, C, 60)
    eps = 1e-4
    s = torch.empty(g.n, dtype=torch.float64, device="cuda")
    st = es.es_single_source(ctx, g, 0, es.make_opts(C, eps, 2024, 0.1), s)
    say(f"  pairs={st.pairs} walk_ms={st.ms_walk:.1f}")
    err = sr.max_error(host(s), S[:, 0])
    assert err <= eps, err


def test_topk_matches_brute_force(es, ctx):
    rng = np.random.default_rng(5)
    for n, k, excl in ((1000, 1, 3), (1000, 999, 0), (100_000, 500, 77), (100_000, 4096, -1), (7, 6, 6)):
        v = np.round(rng.random(n), 3)  # ties
        v[rng.random(n) < 0.3] = 0.0
        say(f"  topk n={n} k={k}")
        idx = torch.empty(k, dtype=torch.int32, device="cuda")
        val = torch.empty(k, dtype=torch.float64, device="cuda")
        es.es_topk(ctx, dev(v, torch.float64), n, excl, k, idx, val)
        ref_i, ref_v = ox.topk(v, excl, k)
        assert np.array_equal(host(idx), ref_i)
        assert np.array_equal(host(val), ref_v)


def test_argument_errors(es, ctx):
    g, og = build_pair(es, ctx, "random_small")
    s = torch.empty(g.n, dtype=torch.float64, device="cuda")
    for u, c, eps, rs in ((-1, C, 1e-3, 1.0), (g.n, C, 1e-3, 1.0), (0, 1.0, 1e-3, 1.0), (0, C, 0.0, 1.0),
                          (0, C, 1e-3, 0.0)):
        with pytest.raises(es.EsError) as e:
            es.es_single_source(ctx, g, u, es.make_opts(c, eps, 1, rs), s)
        assert e.value.status == es.ES_EINVAL
    idx = torch.empty(g.n + 1, dtype=torch.int32, device="cuda")
    with pytest.raises(es.EsError):
        es.es_topk(ctx, s, g.n, 0, g.n, idx, None)
    with pytest.raises(es.EsError) as e:
        es.Graph(ctx, 5, np.array([0, 7]), np.array([1, 2]))
    assert e.value.status == es.ES_EINVAL


def test_allocation_failure_is_reported_and_recoverable(es, ctx):
    """A query whose level storage cannot exist (c = 0.99, eps = 1e-300: about
    6.9e4 levels of 2^20 doubles, 0.58 TB) fails with ES_ENOMEM, and the same
    context then answers an ordinary query."""
    n = 1 << 20
    src, dst = workloads.rmat(n, n, 77)
    g = es.Graph(ctx, n, src, dst)
    s = torch.empty(n, dtype=torch.float64, device="cuda")
    D = torch.ones(n, dtype=torch.float64, device="cuda")  # exact-diagonal mode: no walk budget involved
    L = es.es_num_levels(0.99, 1e-300)
    assert (L + 1) * n * 8 > 400e9
    with pytest.raises(es.EsError) as e:
        es.es_single_source(ctx, g, 0, es.make_opts(0.99, 1e-300, 1, 1.0, d_override=D), s)
    assert e.value.status == es.ES_ENOMEM
    g.close()
    g2, og2 = build_pair(es, ctx, "random_small")
    s2 = torch.empty(g2.n, dtype=torch.float64, device="cuda")
    es.es_single_source(ctx, g2, 3, es.make_opts(C, 1e-3, 1, 1e-3), s2)
    ref = ox.query(og2, 3, C, 1e-3, 1, 1e-3)["s"]
    assert np.abs(host(s2) - ref).max() <= S_TOL


def test_tiny_and_empty_graphs(es, ctx):
    for n, src, dst in ((1, [], []), (3, [], []), (2, [0], [1]), (4, [0, 0, 1], [1, 1, 1])):
        g = es.Graph(ctx, n, np.array(src, dtype=np.int32), np.array(dst, dtype=np.int32))
        og = OracleGraph(n, src, dst)
        for u in range(n):
            s = torch.empty(n, dtype=torch.float64, device="cuda")
            es.es_single_source(ctx, g, u, es.make_opts(C, 1e-3, 1, 1e-3), s)
            ref = ox.query(og, u, C, 1e-3, 1, 1e-3)["s"]
            assert np.abs(host(s) - ref).max() <= S_TOL
