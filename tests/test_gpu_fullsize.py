"""Parity at the full sizes of the standard workloads, in the launch
configurations the benchmark times.

R-MAT n=2^20, m=1.6e7, eps=1e-6, r_scale=1e-5 (the single-source line):
  - every pi^l and pi(k) bit for bit against the oracle (29 levels);
  - every R(k) bit for bit, and the total;
  - M(k) and D^(k) bit for bit on sampled nodes.  Nodes with small R(k) are
    compared directly with the full launch.  On the heaviest nodes (R(k) up
    to about 1.6e10, past 2^32) the oracle simulates the last pairs
    [R(k) - CAP, R(k)), and the full launch must equal head + tail;
  - back-accumulation over all n from a seeded diagonal, within 1e-9;
    then top-500 of that result;
  - the single query equals its five stages run one after another;
  - Algorithm 3 (local deterministic exploitation): l(k), R'(k) and the
    closed-form exact parts bitwise, non-stop walks on sampled nodes and the
    source's last pairs, estimator values, reduced query equal to its stages.

R-MAT n=4.8e6, m=6.9e7 with a block of 64 sources, and the twelve uneven
graphs with 256 sources (the batched lines): every batched answer equals the
one-at-a-time answer for the same query.
"""
import sys

import numpy as np
import pytest
import torch

import workloads
from oracle import exactsim as ox
from oracle.graph import OracleGraph

pytestmark = pytest.mark.gpu

S_TOL = 1e-9
BATCH_TOL = 1e-12          # batched vs single: same arithmetic, other summation order
SINGLE_R_SCALE = 1e-5      # the single-source benchmark line
BATCH_R_SCALE = 1e-7       # the batched benchmark lines
CAP = 4_000_000            # pairs the oracle simulates per heavy node
N_RANDOM = 400


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def host(t):
    return t.cpu().numpy()


def u64(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.uint64)).cuda()


@pytest.fixture(scope="module")
def es():
    from paper_2004_03493_amd import binding
    return binding


@pytest.fixture(scope="module")
def ctx(es):
    c = es.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def rmat1m(es, ctx):
    wl = workloads.RMAT_1M
    say(f"[graph {wl.name}]")
    src, dst = wl.graph()
    g = es.Graph(ctx, wl.n, src, dst)
    og = OracleGraph(wl.n, src, dst)
    return wl, g, og, wl.sources(dst)


@pytest.mark.parametrize("which", [0, 7])
def test_rmat1m_single_source_stages(es, ctx, rmat1m, which):
    wl, g, og, sources = rmat1m
    u = int(sources[which])
    c, eps = wl.c, wl.eps
    L = ox.num_levels(c, eps)
    say(f"  u={u} L={L} forward")
    lv = torch.empty((L + 1) * g.n, dtype=torch.float64, device="cuda")
    pi = torch.empty(g.n, dtype=torch.float64, device="cuda")
    es.es_forward(ctx, g, u, c, L, lv, pi)
    ref_lv, ref_pi = ox.forward_levels(og, u, c, L)
    assert np.array_equal(host(lv).view(np.uint64), ref_lv.reshape(-1).view(np.uint64))
    assert np.array_equal(host(pi).view(np.uint64), ref_pi.view(np.uint64))

    say("  budget")
    R = ox.total_samples(g.n, c, eps, SINGLE_R_SCALE)
    Rk = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    tot = es.es_budget(ctx, g, pi, R, es.ES_ALLOC_PI2, True, Rk, want_total=True)
    ref_R = ox.budget(ref_pi, og.din, R, True)
    assert np.array_equal(host(Rk), ref_R)
    assert tot == int(ref_R.sum())

    say(f"  walks: {tot} pairs, max R(k) {int(ref_R.max())}")
    M = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    es.es_walk_pairs(ctx, g, None, Rk, wl.seed_walk, c, M)
    gM = host(M)
    rng = np.random.default_rng(1000 + which)
    active = np.flatnonzero(ref_R > 0)
    heavy = active[np.argsort(-ref_R[active].astype(np.float64), kind="stable")[:8]]
    light_pool = np.setdiff1d(active[ref_R[active] <= CAP], heavy)
    light = rng.choice(light_pool, size=min(N_RANDOM, len(light_pool)), replace=False)
    # light nodes: the full launch against the oracle
    R_light = np.zeros(g.n, dtype=np.uint64)
    R_light[light] = ref_R[light]
    ref_M_light = ox.walk_counts(og, R_light, wl.seed_walk, c)
    assert np.array_equal(gM[light], ref_M_light[light])
    # heavy nodes: oracle on the tail [R(k) - CAP, R(k)), head + tail = full
    big = heavy[ref_R[heavy] > CAP]
    assert ref_R[big].max() > 2 ** 32, "the heaviest node should take pair indices past 2^32"
    R_hi = np.zeros(g.n, dtype=np.uint64)
    R_hi[big] = ref_R[big]
    R_lo = np.zeros(g.n, dtype=np.uint64)
    R_lo[big] = ref_R[big] - np.uint64(CAP)
    ref_tail = ox.walk_counts(og, R_hi, wl.seed_walk, c, r_begin=R_lo)
    tail = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    head = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    es.es_walk_pairs(ctx, g, u64(R_lo), u64(R_hi), wl.seed_walk, c, tail)
    es.es_walk_pairs(ctx, g, None, u64(R_lo), wl.seed_walk, c, head)
    assert np.array_equal(host(tail)[big], ref_tail[big])
    assert np.array_equal(host(head)[big] + host(tail)[big], gM[big])
    say(f"  {len(light)} light nodes, {len(big)} heavy tails match")

    say("  diagonal")
    D = torch.empty(g.n, dtype=torch.float64, device="cuda")
    es.es_diag(ctx, g, Rk, M, c, True, D)
    gD = host(D)
    ref_D_light = ox.diag_estimate(ref_R[light], ref_M_light[light], og.din[light], c, True)
    assert np.array_equal(gD[light].view(np.uint64), ref_D_light.view(np.uint64))
    exact = og.din <= 1
    assert np.array_equal(gD[exact], np.where(og.din[exact] == 0, 1.0, 1.0 - c))

    say("  back-accumulation from a seeded diagonal")
    drng = np.random.default_rng(2000 + which)
    D_seed = drng.uniform(1.0 - c, 1.0, g.n)
    D_seed[og.din == 0] = 1.0
    D_seed[og.din == 1] = 1.0 - c
    s = torch.empty(g.n, dtype=torch.float64, device="cuda")
    es.es_backward(ctx, g, lv, L, torch.as_tensor(D_seed).cuda(), c, s)
    ref_s = ox.back_accumulate(og, ref_lv, D_seed, c)
    err = np.abs(host(s) - ref_s).max()
    say(f"  max |s - s_ref| = {err:.2e}")
    assert err <= S_TOL

    k = 500
    idx = torch.empty(k, dtype=torch.int32, device="cuda")
    val = torch.empty(k, dtype=torch.float64, device="cuda")
    es.es_topk(ctx, s, g.n, u, k, idx, val)
    ref_idx, ref_val = ox.topk(ref_s, u, k)
    gi, gv = host(idx), host(val)
    assert np.all(np.abs(gv - ref_val) <= S_TOL)
    # sets agree except for ids tied with the k-th value within 2 tol
    edge = ref_val[-1]
    differ = set(gi.tolist()) ^ set(ref_idx.tolist())
    assert all(abs(ref_s[j] - edge) <= 2 * S_TOL for j in differ)

    say("  single query = its stages")
    s_q = torch.empty(g.n, dtype=torch.float64, device="cuda")
    st = es.es_single_source(ctx, g, u, es.make_opts(c, eps, wl.seed_walk, SINGLE_R_SCALE), s_q)
    s_st = torch.empty(g.n, dtype=torch.float64, device="cuda")
    es.es_backward(ctx, g, lv, L, D, c, s_st)
    assert st.pairs == tot
    assert st.meets == int(gM.sum())
    assert torch.equal(s_q, s_st)


def _batch_vs_single(es, ctx, graphs, goq, sources, eps, c, seed, sparse_eps=0.0):
    opts = es.make_opts(c, eps, seed, BATCH_R_SCALE, sparse_eps=sparse_eps)
    outs = [torch.empty(graphs[gi].n, dtype=torch.float64, device="cuda") for gi in goq]
    st = es.es_batch(ctx, graphs, goq, sources, opts, outs, use_hip_graph=True)
    say(f"  batch of {len(sources)}: {st.pairs} pairs, {st.level_bytes / 1e9:.2f} GB of levels")
    one = torch.empty(max(g.n for g in graphs), dtype=torch.float64, device="cuda")
    worst = 0.0
    for q, (gi, u) in enumerate(zip(goq, sources)):
        n = graphs[gi].n
        es.es_single_source(ctx, graphs[gi], u, opts, one[:n])
        worst = max(worst, float((outs[q] - one[:n]).abs().max()))
    say(f"  max |batched - single| = {worst:.2e}")
    assert worst <= BATCH_TOL


@pytest.mark.parametrize("sparse_eps", [0.0, 1e-6])
def test_rmat4m8_block64_equals_single_source(es, ctx, sparse_eps):
    """Dense levels, and sparse linearization at eps_s = eps (every source keeps
    exactly the entries its single-source query keeps)."""
    wl = workloads.RMAT_4M8
    say(f"[graph {wl.name}]")
    src, dst = wl.graph()
    g = es.Graph(ctx, wl.n, src, dst)
    sources = [int(x) for x in wl.sources(dst)]
    _batch_vs_single(es, ctx, [g], [0] * len(sources), sources, wl.eps, wl.c, wl.seed_walk, sparse_eps)


def test_uneven_twelve_graphs_equal_single_source(es, ctx):
    wl = workloads.UNEVEN_12
    say(f"[graphs {wl.name}]")
    counts = workloads.uneven_source_counts(len(wl.parts), wl.num_sources, wl.seed_src)
    graphs, goq, sources = [], [], []
    for gi, part in enumerate(wl.parts):
        src, dst = part.graph()
        graphs.append(es.Graph(ctx, part.n, src, dst))
        s = workloads.pick_sources(part.n, dst, int(counts[gi]), wl.seed_src + gi)
        sources += [int(x) for x in s]
        goq += [gi] * len(s)
    _batch_vs_single(es, ctx, graphs, goq, sources, wl.eps, wl.c, wl.seed_walk)


def _lde_full(es, ctx, g, og, u, c, eps, r_scale, seed, ref_pi, lv, L):
    """Algorithm 3 at full size: plan (l(k), R'(k), closed-form sums) bitwise
    against the oracle, non-stop walks on sampled nodes and the source's last
    pairs, estimator values, and the reduced query equal to its stages."""
    from oracle import lde
    R = ox.total_samples(g.n, c, eps, r_scale)
    Rk = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    es.es_budget(ctx, g, torch.as_tensor(ref_pi).cuda(), R, es.ES_ALLOC_PI2, True, Rk)
    ref_R = ox.budget(ref_pi, og.din, R, True)
    assert np.array_equal(host(Rk), ref_R)
    others = np.arange(g.n) != u
    plans = {}
    # Lemma 4 on the CPU for the source where the sparse-matrix oracle holds the graph
    znodes = [u] if hasattr(og, "PT") else []
    for mode in (1, 2):
        ell = torch.empty(g.n, dtype=torch.int32, device="cuda")
        zsum = torch.empty(g.n, dtype=torch.float64, device="cuda")
        R2 = torch.empty(g.n, dtype=torch.uint64, device="cuda")
        es.es_lde_plan(ctx, g, Rk, c, mode, 3, ell, zsum, R2)
        r_ell, r_z, r_R2 = lde.plan(og, ref_R, c, mode, max_level=3, zsum_nodes=znodes if mode == 1 else [])
        assert np.array_equal(host(ell), r_ell)
        assert np.array_equal(host(R2), r_R2)
        gz = host(zsum)
        shallow = r_ell <= 1
        assert np.array_equal(gz[shallow].view(np.uint64), r_z[shallow].view(np.uint64))
        deep = np.flatnonzero(r_ell >= 2)
        assert np.all((gz[deep] > 0.0) & (gz[deep] < 1.0))
        if mode == 1 and znodes and r_ell[u] >= 2:
            assert abs(gz[u] - r_z[u]) <= 1e-13, (gz[u], r_z[u])
        plans[mode] = (ell, zsum, R2, r_ell, r_z, r_R2)
    ell, zsum, R2, r_ell, r_z, r_R2 = plans[2]
    say(f"  l(u)={int(r_ell[u])} zsum(u)={host(zsum)[u]:.6g} pairs {int(r_R2.sum())} (plain {int(ref_R.sum())}); "
        f"{int((r_ell >= 2).sum())} nodes with l >= 2, {int((r_ell == 3).sum())} with l = 3")
    M = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    es.es_walk_pairs_lde(ctx, g, None, R2, ell, seed, c, M)
    gM = host(M)
    rng = np.random.default_rng(77)
    pool = np.flatnonzero(others & (r_R2 > 0) & (r_R2 <= CAP))
    light = rng.choice(pool, size=min(N_RANDOM, len(pool)), replace=False)
    R_light = np.zeros(g.n, dtype=np.uint64)
    R_light[light] = r_R2[light]
    ref_M = ox.walk_counts(og, R_light, seed, c, nonstop=r_ell)
    assert np.array_equal(gM[light], ref_M[light])
    if r_R2[u] > CAP:
        lo = np.zeros(g.n, dtype=np.uint64)
        hi = np.zeros(g.n, dtype=np.uint64)
        lo[u], hi[u] = r_R2[u] - np.uint64(CAP), r_R2[u]
        tail = torch.empty(g.n, dtype=torch.uint64, device="cuda")
        head = torch.empty(g.n, dtype=torch.uint64, device="cuda")
        es.es_walk_pairs_lde(ctx, g, u64(lo), u64(hi), ell, seed, c, tail)
        es.es_walk_pairs_lde(ctx, g, None, u64(lo), ell, seed, c, head)
        assert host(tail)[u] == ox.walk_counts(og, hi, seed, c, r_begin=lo, nonstop=r_ell)[u]
        assert host(head)[u] + host(tail)[u] == gM[u]
    D = torch.empty(g.n, dtype=torch.float64, device="cuda")
    es.es_diag_lde(ctx, g, R2, M, ell, zsum, c, True, D)
    # estimator values where the oracle's exact part is bitwise (l <= 1)
    light = light[r_ell[light] <= 1]
    ref_D = lde.diag_estimate(r_R2[light], ref_M[light], r_ell[light], r_z[light], c, og.din[light])
    assert np.array_equal(host(D)[light].view(np.uint64), ref_D.view(np.uint64))
    s_st = torch.empty(g.n, dtype=torch.float64, device="cuda")
    es.es_backward(ctx, g, lv, L, D, c, s_st)
    s_q = torch.empty(g.n, dtype=torch.float64, device="cuda")
    st = es.es_single_source(ctx, g, u, es.make_opts(c, eps, seed, r_scale, lde=2), s_q)
    assert st.pairs == int(r_R2.sum()) and st.lde_source_level == int(r_ell[u])
    assert torch.equal(s_q, s_st)


def test_rmat1m_local_exploitation(es, ctx, rmat1m):
    wl, g, og, sources = rmat1m
    u = int(sources[0])
    L = ox.num_levels(wl.c, wl.eps)
    lv = torch.empty((L + 1) * g.n, dtype=torch.float64, device="cuda")
    pi = torch.empty(g.n, dtype=torch.float64, device="cuda")
    es.es_forward(ctx, g, u, wl.c, L, lv, pi)
    _, ref_pi = ox.forward_levels(og, u, wl.c, L)
    assert np.array_equal(host(pi).view(np.uint64), ref_pi.view(np.uint64))
    _lde_full(es, ctx, g, og, u, wl.c, wl.eps, SINGLE_R_SCALE, wl.seed_walk, ref_pi, lv, L)


def test_rmat1m_sparse_linearization(es, ctx, rmat1m):
    """Sparse linearization (Section 3.2, Lemma 2) at eps_s = eps = 1e-6: the
    kept entries of all levels bit for bit, the back-accumulation from them
    with a seeded diagonal over all n within 1e-9, and the sampled query
    within eps_s below the dense one with the same walks."""
    wl, g, og, sources = rmat1m
    u = int(sources[3])
    c, eps = wl.c, wl.eps
    L = ox.num_levels(c, eps)
    cap = es.es_sparse_capacity(g.n, g.m, L, c, eps)
    idx = torch.empty(cap, dtype=torch.int32, device="cuda")
    val = torch.empty(cap, dtype=torch.float64, device="cuda")
    counts = es.es_forward_sparse(ctx, g, u, c, L, eps, idx, val)
    ref_lv, ref_pi = ox.forward_levels(og, u, c, L)
    theta = ox.sparse_threshold(c, eps)
    gi, gv = host(idx), host(val)
    pos = 0
    for l in range(L + 1):
        want = np.flatnonzero(ref_lv[l] > theta)
        assert counts[l] == len(want), l
        order = np.argsort(gi[pos:pos + counts[l]])
        assert np.array_equal(gi[pos:pos + counts[l]][order], want), l
        assert np.array_equal(gv[pos:pos + counts[l]][order].view(np.uint64), ref_lv[l][want].view(np.uint64)), l
        pos += counts[l]
    say(f"  u={u}: {pos} entries kept of {(L + 1) * g.n} (capacity {cap})")

    kept = ox.sparsify_levels(ref_lv, theta)
    drng = np.random.default_rng(3000)
    D_seed = drng.uniform(1.0 - c, 1.0, g.n)
    D_seed[og.din == 0] = 1.0
    D_seed[og.din == 1] = 1.0 - c
    s = torch.empty(g.n, dtype=torch.float64, device="cuda")
    st = es.es_single_source(ctx, g, u, es.make_opts(c, eps, 1, 1.0, d_override=torch.as_tensor(D_seed).cuda(),
                                                      sparse_eps=eps), s)
    ref_s = ox.back_accumulate(og, kept, D_seed, c)
    err = np.abs(host(s) - ref_s).max()
    say(f"  seeded diagonal: max |s - s_ref| = {err:.2e}, {st.level_bytes / 1e6:.1f} MB of levels")
    assert err <= S_TOL
    assert st.level_entries == pos

    s_d = torch.empty(g.n, dtype=torch.float64, device="cuda")
    st_d = es.es_single_source(ctx, g, u, es.make_opts(c, eps, wl.seed_walk, SINGLE_R_SCALE), s_d)
    st_s = es.es_single_source(ctx, g, u, es.make_opts(c, eps, wl.seed_walk, SINGLE_R_SCALE, sparse_eps=eps), s)
    assert st_s.pairs == st_d.pairs and st_s.meets == st_d.meets
    diff = host(s_d) - host(s)
    say(f"  sampled: dense - sparse in [{diff.min():.2e}, {diff.max():.2e}]; "
        f"levels {st_s.level_bytes / 1e6:.1f} MB vs {st_d.level_bytes / 1e6:.1f} MB dense")
    assert diff.min() >= -1e-12 and diff.max() <= eps
