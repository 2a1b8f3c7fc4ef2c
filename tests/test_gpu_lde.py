"""GPU local deterministic exploitation (Section 3.2, Algorithm 3, Lemma 4)
against the oracle: the level plan (the printed edge-counter rule for every
sampled node, capped or not), the non-stop walk pairs, the estimator, whole
queries, and accuracy against the Power Method."""
import sys

import numpy as np
import pytest
import torch

import workloads
from graphs import diamond, fork, hub_graph, random_graph, three_sources
from oracle import exactsim as ox
from oracle import lde
from oracle import simrank as sr
from oracle.graph import OracleGraph

pytestmark = pytest.mark.gpu

C = 0.6
S_TOL = 1e-9


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def host(t):
    return t.cpu().numpy()


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype).cuda()


@pytest.fixture(scope="module")
def es():
    from paper_2004_03493_amd import binding
    return binding


@pytest.fixture(scope="module")
def ctx(es):
    c = es.Context(0)
    yield c
    c.close()


GRAPHS = {
    "chung_lu_2k": lambda: (2000,) + workloads.chung_lu(2000, 20000, 11),
    "rmat_32k": lambda: (1 << 15,) + workloads.rmat(1 << 15, 500_000, 5),
    "hubs": lambda: hub_graph(30000, 20000, 20000, 60000, 3),
    "random_small": lambda: random_graph(50, 200, 1),
}
_cache = {}


def pair(es, ctx, name):
    if name not in _cache:
        n, s, d = GRAPHS[name]()
        say(f"[graph {name}]")
        _cache[name] = (es.Graph(ctx, n, s, d), OracleGraph(n, s, d))
    return _cache[name]


def stages(es, ctx, g, og, u, eps, r_scale):
    """GPU forward levels and budget, with the oracle's own (bitwise equal)."""
    L = ox.num_levels(C, eps)
    lv = torch.empty((L + 1) * g.n, dtype=torch.float64, device="cuda")
    pi = torch.empty(g.n, dtype=torch.float64, device="cuda")
    es.es_forward(ctx, g, u, C, L, lv, pi)
    R = ox.total_samples(g.n, C, eps, r_scale)
    Rk = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    es.es_budget(ctx, g, pi, R, es.ES_ALLOC_PI2, True, Rk)
    ref_lv, ref_pi = ox.forward_levels(og, u, C, L)
    ref_R = ox.budget(ref_pi, og.din, R, True)
    assert np.array_equal(host(Rk), ref_R)
    return L, lv, Rk, ref_lv, ref_R


def gpu_plan(es, ctx, g, Rk, mode, cap=3):
    ell = torch.empty(g.n, dtype=torch.int32, device="cuda")
    zsum = torch.empty(g.n, dtype=torch.float64, device="cuda")
    R2 = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    es.es_lde_plan(ctx, g, Rk, C, mode, cap, ell, zsum, R2)
    return ell, zsum, R2


def check_plan(og, got, ref_R, mode, cap, u, zmax=40):
    """GPU plan against the oracle: levels and counts bit for bit, the exact
    part bit for bit at one level (c/d_in) and within 1e-13 deeper (Lemma 4,
    on the source and on up to zmax other deep nodes)."""
    ell, zsum, R2 = (host(t) for t in got)
    r_ell = lde.plan(og, ref_R, C, mode, max_level=cap, zsum_nodes=[])[0]
    deep = np.flatnonzero(r_ell >= 2)
    pick = [int(k) for k in deep if k == u] + [int(k) for k in deep if k != u][:zmax]
    r_ell, r_z, r_R2 = lde.plan(og, ref_R, C, mode, max_level=cap, zsum_nodes=pick)
    assert np.array_equal(ell, r_ell)
    assert np.array_equal(R2, r_R2)
    shallow = r_ell <= 1
    assert np.array_equal(zsum[shallow].view(np.uint64), r_z[shallow].view(np.uint64))
    for k in pick:
        assert abs(zsum[k] - r_z[k]) <= 1e-13 * max(1.0, abs(r_z[k])), (k, r_ell[k], zsum[k], r_z[k])
    return r_ell, len(deep)


@pytest.mark.parametrize("name", list(GRAPHS))
def test_plan_matches_oracle(es, ctx, name):
    g, og = pair(es, ctx, name)
    for u in sorted({int(np.argmax(og.din)), int(np.argsort(og.din)[len(og.din) // 2]), 3}):
        for r_scale in (1e-6, 1e-3, 1e-1):
            L, lv, Rk, _, ref_R = stages(es, ctx, g, og, u, 1e-4, r_scale)
            for mode in (lde.MODE_OFF, lde.MODE_AS_PRINTED, lde.MODE_REDUCED):
                for cap in ((1, 2, 3) if mode == lde.MODE_AS_PRINTED else (3,)):
                    got = gpu_plan(es, ctx, g, Rk, mode, cap)
                    r_ell, ndeep = check_plan(og, got, ref_R, mode, cap, u)
            say(f"  u={u} r_scale={r_scale:g}: l(u)={int(r_ell[u])}, {ndeep} nodes with l >= 2, "
                f"{int((r_ell == 3).sum())} with l = 3")


def test_plan_uncapped(es, ctx):
    """The printed rule without a cap: where it asks for more than three
    levels the call is refused; where it stays within three (or the rounds
    run dry) the plan equals the oracle's."""
    g, og = pair(es, ctx, "chung_lu_2k")
    u = int(np.argmax(og.din))
    for r_scale in (1e-6, 1e-4, 1e-2, 1.0):
        L, lv, Rk, _, ref_R = stages(es, ctx, g, og, u, 1e-4, r_scale)
        r4 = lde.plan(og, ref_R, C, lde.MODE_AS_PRINTED, max_level=4, zsum_nodes=[])[0]
        if r4.max() >= 4:
            with pytest.raises(es.EsError) as e:
                gpu_plan(es, ctx, g, Rk, lde.MODE_AS_PRINTED, 0)
            assert e.value.status == es.ES_EUNSUPPORTED
            say(f"  r_scale={r_scale:g}: {int((r4 >= 4).sum())} nodes need 4+ levels: refused")
        else:
            got = gpu_plan(es, ctx, g, Rk, lde.MODE_AS_PRINTED, 0)
            check_plan(og, got, ref_R, lde.MODE_AS_PRINTED, 4, u)
            say(f"  r_scale={r_scale:g}: uncapped plan, l(u)={int(r4[u])}")
    # graphs whose rounds run dry take their exact level whatever the budget
    for mk in (fork, three_sources, diamond):
        n, s_, d_ = mk()
        g2 = es.Graph(ctx, n, s_, d_)
        og2 = OracleGraph(n, s_, d_)
        R = np.zeros(n, dtype=np.uint64)
        R[0] = 10 ** 12
        ell, zsum, _ = gpu_plan(es, ctx, g2, dev(R, torch.uint64), lde.MODE_AS_PRINTED, 3)
        ref = lde.printed_exploitation(og2, 0, C, lde.edge_budget(R, C)[0], cap=3)
        assert int(host(ell)[0]) == ref[0]
        assert abs(host(zsum)[0] - sum(ref[1])) <= 1e-15
        g2.close()


def test_plan_cache_gives_the_same_bits(es, ctx):
    """The per-graph cache of table sums: a plan on a graph that has answered
    other queries equals, bit for bit, the plan on a fresh handle of the same
    edges, for every source order."""
    n, s_, d_ = GRAPHS["hubs"]()
    og = OracleGraph(n, s_, d_)
    us = [int(x) for x in np.argsort(-og.din)[:3]] + [7]
    ga = es.Graph(ctx, n, s_, d_)
    plans = {}
    for u in us:  # warm: each plan after the previous ones filled the cache
        L, lv, Rk, _, _ = stages(es, ctx, ga, og, u, 1e-4, 1e-1)
        plans[u] = [host(t).copy() for t in gpu_plan(es, ctx, ga, Rk, lde.MODE_REDUCED)]
    ga.close()
    for u in reversed(us):  # cold: a new handle per source
        gb = es.Graph(ctx, n, s_, d_)
        L, lv, Rk, _, _ = stages(es, ctx, gb, og, u, 1e-4, 1e-1)
        cold = [host(t) for t in gpu_plan(es, ctx, gb, Rk, lde.MODE_REDUCED)]
        for a, b in zip(plans[u], cold):
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), u
        say(f"  u={u}: {int((cold[0] >= 2).sum())} nodes with l >= 2, warm = cold")
        gb.close()


@pytest.mark.parametrize("name", ["chung_lu_2k", "rmat_32k", "hubs"])
def test_nonstop_walks_bitwise(es, ctx, name):
    g, og = pair(es, ctx, name)
    rng = np.random.default_rng(8)
    R = rng.integers(0, 500, g.n).astype(np.uint64)
    R[rng.random(g.n) < 0.3] = 0
    R[int(np.argmax(og.din))] = 200_000
    ell = rng.integers(0, 4, g.n).astype(np.int32)
    M = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    es.es_walk_pairs_lde(ctx, g, None, dev(R, torch.uint64), dev(ell, torch.int32), 41, C, M)
    assert np.array_equal(host(M), ox.walk_counts(og, R, 41, C, nonstop=ell))
    # ranges split like the plain pairs
    lo = (R // 3).astype(np.uint64)
    Ma = torch.empty_like(M)
    Mb = torch.empty_like(M)
    es.es_walk_pairs_lde(ctx, g, None, dev(lo, torch.uint64), dev(ell, torch.int32), 41, C, Ma)
    es.es_walk_pairs_lde(ctx, g, dev(lo, torch.uint64), dev(R, torch.uint64), dev(ell, torch.int32), 41, C, Mb)
    assert np.array_equal(host(Ma) + host(Mb), host(M))
    # l = 0 everywhere is Algorithm 2
    M0 = torch.empty_like(M)
    es.es_walk_pairs(ctx, g, None, dev(R, torch.uint64), 41, C, M0)
    es.es_walk_pairs_lde(ctx, g, None, dev(R, torch.uint64), dev(np.zeros(g.n, np.int32), torch.int32), 41, C, Ma)
    assert torch.equal(M0, Ma)


def test_diag_lde_bitwise(es, ctx):
    g, og = pair(es, ctx, "chung_lu_2k")
    rng = np.random.default_rng(9)
    R = rng.integers(0, 1000, g.n).astype(np.uint64)
    M = (R.astype(np.float64) * rng.uniform(0, 0.5, g.n)).astype(np.uint64)
    ell = rng.integers(0, 4, g.n).astype(np.int32)
    zsum = rng.uniform(0, 0.3, g.n)
    for small in (True, False):
        D = torch.empty(g.n, dtype=torch.float64, device="cuda")
        es.es_diag_lde(ctx, g, dev(R, torch.uint64), dev(M, torch.uint64), dev(ell, torch.int32),
                       dev(zsum, torch.float64), C, small, D)
        ref = lde.diag_estimate(R, M, ell, zsum, C, og.din, small)
        assert np.array_equal(host(D).view(np.uint64), ref.view(np.uint64))


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("name", ["chung_lu_2k", "rmat_32k"])
def test_single_source_equals_stages_and_oracle(es, ctx, name, mode):
    g, og = pair(es, ctx, name)
    u = int(np.argmax(og.din))
    eps, r_scale, seed = 1e-4, 1e-3, 77
    L, lv, Rk, ref_lv, ref_R = stages(es, ctx, g, og, u, eps, r_scale)
    ell, zsum, R2 = gpu_plan(es, ctx, g, Rk, mode)
    M = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    es.es_walk_pairs_lde(ctx, g, None, R2, ell, seed, C, M)
    D = torch.empty(g.n, dtype=torch.float64, device="cuda")
    es.es_diag_lde(ctx, g, R2, M, ell, zsum, C, True, D)
    s_st = torch.empty(g.n, dtype=torch.float64, device="cuda")
    es.es_backward(ctx, g, lv, L, D, C, s_st)
    s_q = torch.empty(g.n, dtype=torch.float64, device="cuda")
    st = es.es_single_source(ctx, g, u, es.make_opts(C, eps, seed, r_scale, lde=mode), s_q)
    assert torch.equal(s_q, s_st)
    assert st.pairs == int(host(R2).sum())
    assert st.lde_source_level == int(host(ell)[u])
    # the oracle end to end
    r_ell, r_z, r_R2 = lde.plan(og, ref_R, C, mode)
    r_M = ox.walk_counts(og, r_R2, seed, C, nonstop=r_ell)
    assert np.array_equal(host(M), r_M)
    r_D = lde.diag_estimate(r_R2, r_M, r_ell, r_z, C, og.din)
    r_s = ox.back_accumulate(og, ref_lv, r_D, C)
    err = np.abs(host(s_q) - r_s).max()
    say(f"  l(u)={st.lde_source_level} zsum(u)={st.lde_source_zsum:.6g} pairs {st.pairs} "
        f"(plain {int(ref_R.sum())}) max|s - oracle| {err:.1e}, {int((r_ell >= 2).sum())} nodes with l >= 2")
    assert err <= S_TOL
    assert abs(st.lde_source_zsum - r_z[u]) <= 1e-13
    assert np.abs(host(zsum) - r_z).max() <= 1e-13


def test_accuracy_against_power_method(es, ctx):
    """Algorithm 3 as printed lowers MaxError at equal pairs; the reduced
    sample count keeps MaxError near Algorithm 2's with fewer pairs."""
    g, og = pair(es, ctx, "chung_lu_2k")
    S = sr.power_method(og, C, 60)
    s = torch.empty(g.n, dtype=torch.float64, device="cuda")
    eps = 1e-4
    err = {0: [], 1: [], 2: []}
    pairs = {0: 0, 1: 0, 2: 0}
    for u in (0, 5, 50, 300):
        for seed in range(6):
            for mode in (0, 1, 2):
                st = es.es_single_source(ctx, g, u, es.make_opts(C, eps, 500 + seed, 1e-3, lde=mode), s)
                err[mode].append(sr.max_error(host(s), S[:, u]))
                pairs[mode] += st.pairs
    m = {k: float(np.mean(v)) for k, v in err.items()}
    say(f"  MaxError plain {m[0]:.3e} as printed {m[1]:.3e} reduced {m[2]:.3e}; "
        f"pairs {pairs[0]} {pairs[1]} {pairs[2]}")
    assert pairs[1] == pairs[0]
    assert pairs[2] < 0.8 * pairs[0]
    assert m[1] < m[0]
    assert m[2] <= 1.5 * m[0]
    assert max(err[2]) <= eps


def _oracle_lde_query(og, u, eps, seed, r_scale, mode):
    L = ox.num_levels(C, eps)
    lv, pi = ox.forward_levels(og, u, C, L)
    R = ox.total_samples(og.n, C, eps, r_scale)
    Rk = ox.budget(pi, og.din, R, True)
    ell, z, R2 = lde.plan(og, Rk, C, mode)
    M = ox.walk_counts(og, R2, seed, C, nonstop=ell)
    return ox.back_accumulate(og, lv, lde.diag_estimate(R2, M, ell, z, C, og.din), C)


def test_tiny_graphs_and_small_l(es, ctx):
    """Empty and tiny graphs, sources without in-neighbours, and eps = 0.9
    (L = 2: the exact levels do not depend on L)."""
    cases = [(1, [], []), (3, [], []), (2, [0], [1]), (4, [0, 0, 1], [1, 1, 1]),
             (5, [1, 2, 3, 4, 2, 3], [0, 0, 0, 0, 1, 1]), (6, [0, 1, 2, 3, 4, 5], [1, 2, 3, 4, 5, 0])]
    for n, src, dst in cases:
        g = es.Graph(ctx, n, np.array(src, dtype=np.int32), np.array(dst, dtype=np.int32))
        og = OracleGraph(n, src, dst)
        s = torch.empty(n, dtype=torch.float64, device="cuda")
        for u in range(n):
            for eps in (1e-3, 0.9):
                for mode in (1, 2):
                    es.es_single_source(ctx, g, u, es.make_opts(C, eps, 3, 1e-2, lde=mode), s)
                    ref = _oracle_lde_query(og, u, eps, 3, 1e-2, mode)
                    assert np.abs(host(s) - ref).max() <= S_TOL, (n, u, eps, mode)


def test_lde_argument_errors(es, ctx):
    g, og = pair(es, ctx, "random_small")
    s = torch.empty(g.n, dtype=torch.float64, device="cuda")
    with pytest.raises(es.EsError) as e:
        es.es_single_source(ctx, g, 0, es.make_opts(C, 1e-3, 1, 1e-3, lde=3), s)
    assert e.value.status == es.ES_EINVAL
    Rk = torch.zeros(g.n, dtype=torch.uint64, device="cuda")
    ell = torch.empty(g.n, dtype=torch.int32, device="cuda")
    z = torch.empty(g.n, dtype=torch.float64, device="cuda")
    R2 = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    for c, mode in ((1.5, 1), (0.0, 1), (C, 5), (C, -1)):
        with pytest.raises(es.EsError) as e:
            es.es_lde_plan(ctx, g, Rk, c, mode, 3, ell, z, R2)
        assert e.value.status == es.ES_EINVAL
    # an uncapped query whose rule asks for more than three exact levels
    g2, og2 = pair(es, ctx, "chung_lu_2k")
    s2 = torch.empty(g2.n, dtype=torch.float64, device="cuda")
    with pytest.raises(es.EsError) as e:
        es.es_single_source(ctx, g2, 0, es.make_opts(C, 1e-4, 1, 1.0, lde=1, lde_max_level=0), s2)
    assert e.value.status == es.ES_EUNSUPPORTED
    # the context stays usable
    es.es_single_source(ctx, g2, 0, es.make_opts(C, 1e-4, 1, 1e-4, lde=1), s2)
    # batches run Algorithm 2 only
    outs = [torch.empty(g.n, dtype=torch.float64, device="cuda")]
    with pytest.raises(es.EsError) as e:
        es.es_batch(ctx, [g], [0], [0], es.make_opts(C, 1e-3, 1, 1e-3, lde=1), outs)
    assert e.value.status == es.ES_EUNSUPPORTED
