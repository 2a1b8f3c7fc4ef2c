"""Parity on the largest workload: R-MAT n=4.2e7, m=1.4e9, eps=1e-6.

The sparse-matrix oracle cannot hold this graph, so the CSR oracle (plain C
loops, pinned against the sparse-matrix oracle on small graphs) computes the
linear passes here.  Checked:
  - every pi^l and pi(k) bit for bit (29 levels, 42 million nodes);
  - every R(k) bit for bit under the pi^2 allocation;
  - M(k) and D^(k) bit for bit on sampled nodes: small R(k) directly, the
    heaviest nodes on the tail [R(k) - CAP, R(k)) with head + tail = full;
  - back-accumulation over all n from a seeded diagonal within 1e-9, top-500;
  - the single query equals its stages, for the pi^2 and the learned
    allocation; learned features on sampled nodes, and the weighted budget
    bit for bit from a seeded variance vector.
"""
import sys
import time

import numpy as np
import pytest
import torch

import workloads
from oracle import csr
from oracle import exactsim as ox
from oracle import mlp

pytestmark = pytest.mark.gpu

S_TOL = 1e-9
R_SCALE = 1e-5
CAP = 4_000_000
N_RANDOM = 400
T0 = time.time()


def say(msg):
    print(f"  [{time.time() - T0:6.1f}s] {msg}", flush=True)
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
def big(es, ctx):
    wl = workloads.RMAT_42M
    say(f"generating {wl.name}")
    src, dst = wl.graph()
    say("graph on the device")
    g = es.Graph(ctx, wl.n, src, dst)
    assert g.m == wl.m
    say("CSR oracle graph")
    cg = csr.CsrGraph(wl.n, src, dst)
    u = int(wl.sources(dst)[0])
    del src, dst
    L = ox.num_levels(wl.c, wl.eps)
    say(f"GPU forward u={u} L={L}")
    lv = torch.empty((L + 1) * g.n, dtype=torch.float64, device="cuda")
    pi = torch.empty(g.n, dtype=torch.float64, device="cuda")
    es.es_forward(ctx, g, u, wl.c, L, lv, pi)
    torch.cuda.synchronize()
    say("oracle forward")
    ref_lv, ref_pi = csr.forward_levels(cg, u, wl.c, L)
    say("ready")
    return dict(wl=wl, g=g, cg=cg, u=u, L=L, lv=lv, pi=pi, ref_lv=ref_lv, ref_pi=ref_pi)


def test_forward_bitwise(big):
    lv, ref_lv, L, n = big["lv"], big["ref_lv"], big["L"], big["g"].n
    for l in range(L + 1):
        got = host(lv[l * n:(l + 1) * n])
        assert np.array_equal(got.view(np.uint64), ref_lv[l].view(np.uint64)), f"level {l}"
    assert np.array_equal(host(big["pi"]).view(np.uint64), big["ref_pi"].view(np.uint64))


def _budget(es, ctx, big):
    wl, g = big["wl"], big["g"]
    R = ox.total_samples(g.n, wl.c, wl.eps, R_SCALE)
    Rk = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    tot = es.es_budget(ctx, g, big["pi"], R, es.ES_ALLOC_PI2, True, Rk, want_total=True)
    return R, Rk, tot


def test_budget_walks_diag(es, ctx, big):
    wl, g, cg = big["wl"], big["g"], big["cg"]
    c = wl.c
    R, Rk, tot = _budget(es, ctx, big)
    ref_R = ox.budget(big["ref_pi"], cg.din, R, True)
    assert np.array_equal(host(Rk), ref_R)
    assert tot == int(ref_R.sum())
    say(f"walks: {tot} pairs, max R(k) {int(ref_R.max())}")
    M = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    es.es_walk_pairs(ctx, g, None, Rk, wl.seed_walk, c, M)
    gM = host(M)
    rng = np.random.default_rng(4242)
    active = np.flatnonzero(ref_R > 0)
    heavy = active[np.argsort(-ref_R[active].astype(np.float64), kind="stable")[:8]]
    light_pool = np.setdiff1d(active[ref_R[active] <= CAP], heavy)
    light = rng.choice(light_pool, size=min(N_RANDOM, len(light_pool)), replace=False)
    R_light = np.zeros(g.n, dtype=np.uint64)
    R_light[light] = ref_R[light]
    ref_M_light = ox.walk_counts(cg, R_light, wl.seed_walk, c)
    assert np.array_equal(gM[light], ref_M_light[light])
    bign = heavy[ref_R[heavy] > CAP]
    R_hi = np.zeros(g.n, dtype=np.uint64)
    R_hi[bign] = ref_R[bign]
    R_lo = np.zeros(g.n, dtype=np.uint64)
    R_lo[bign] = ref_R[bign] - np.uint64(CAP)
    ref_tail = ox.walk_counts(cg, R_hi, wl.seed_walk, c, r_begin=R_lo)
    tail = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    head = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    es.es_walk_pairs(ctx, g, u64(R_lo), u64(R_hi), wl.seed_walk, c, tail)
    es.es_walk_pairs(ctx, g, None, u64(R_lo), wl.seed_walk, c, head)
    assert np.array_equal(host(tail)[bign], ref_tail[bign])
    assert np.array_equal(host(head)[bign] + host(tail)[bign], gM[bign])
    say(f"{len(light)} light nodes, {len(bign)} heavy tails match")
    D = torch.empty(g.n, dtype=torch.float64, device="cuda")
    es.es_diag(ctx, g, Rk, M, c, True, D)
    gD = host(D)
    ref_D_light = ox.diag_estimate(ref_R[light], ref_M_light[light], cg.din[light], c, True)
    assert np.array_equal(gD[light].view(np.uint64), ref_D_light.view(np.uint64))
    exact = cg.din <= 1
    assert np.array_equal(gD[exact], np.where(cg.din[exact] == 0, 1.0, 1.0 - c))


def test_backward_and_topk(es, ctx, big):
    wl, g, cg, u, L = big["wl"], big["g"], big["cg"], big["u"], big["L"]
    c = wl.c
    rng = np.random.default_rng(4343)
    D_seed = rng.uniform(1.0 - c, 1.0, g.n)
    D_seed[cg.din == 0] = 1.0
    D_seed[cg.din == 1] = 1.0 - c
    s = torch.empty(g.n, dtype=torch.float64, device="cuda")
    es.es_backward(ctx, g, big["lv"], L, torch.as_tensor(D_seed).cuda(), c, s)
    say("oracle back-accumulation")
    ref_s = csr.back_accumulate(cg, big["ref_lv"], D_seed, c)
    gs = host(s)
    err = np.abs(gs - ref_s).max()
    say(f"max |s - s_ref| = {err:.2e}")
    assert err <= S_TOL
    k = 500
    idx = torch.empty(k, dtype=torch.int32, device="cuda")
    val = torch.empty(k, dtype=torch.float64, device="cuda")
    es.es_topk(ctx, s, g.n, u, k, idx, val)
    ref_idx, ref_val = ox.topk(ref_s, u, k)
    assert np.all(np.abs(host(val) - ref_val) <= S_TOL)
    differ = set(host(idx).tolist()) ^ set(ref_idx.tolist())
    assert all(abs(ref_s[j] - ref_val[-1]) <= 2 * S_TOL for j in differ)


def test_single_query_equals_stages(es, ctx, big):
    wl, g, u, L = big["wl"], big["g"], big["u"], big["L"]
    c = wl.c
    R, Rk, tot = _budget(es, ctx, big)
    M = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    es.es_walk_pairs(ctx, g, None, Rk, wl.seed_walk, c, M)
    D = torch.empty(g.n, dtype=torch.float64, device="cuda")
    es.es_diag(ctx, g, Rk, M, c, True, D)
    s_st = torch.empty(g.n, dtype=torch.float64, device="cuda")
    es.es_backward(ctx, g, big["lv"], L, D, c, s_st)
    s_q = torch.empty(g.n, dtype=torch.float64, device="cuda")
    st = es.es_single_source(ctx, g, u, es.make_opts(c, wl.eps, wl.seed_walk, R_SCALE), s_q)
    say(f"query: {st.pairs} pairs, walk {st.ms_walk:.1f} ms, forward {st.ms_forward:.1f} ms, "
        f"backward {st.ms_backward:.1f} ms")
    assert st.pairs == tot
    assert torch.equal(s_q, s_st)


def test_learned_allocation(es, ctx, big):
    wl, g, cg, u, L = big["wl"], big["g"], big["cg"], big["u"], big["L"]
    c = wl.c
    F = torch.empty((g.n, mlp.NF), dtype=torch.float32, device="cuda")
    es.es_mlp_features(ctx, g, c, F)
    rng = np.random.default_rng(4444)
    nodes = np.unique(np.concatenate([rng.integers(0, g.n, 2000), np.argsort(-cg.din)[:50]]))
    ref_F = mlp.features_at(cg, c, nodes)
    got = host(F)[nodes].astype(np.float64)
    assert np.all(np.abs(got - ref_F) <= 2e-6 * (1 + np.abs(ref_F)))
    say("features match on sampled nodes")
    # weighted allocation from a seeded variance vector, every node
    R = ox.total_samples(g.n, c, wl.eps, R_SCALE)
    v = rng.uniform(1e-6, 0.25, g.n).astype(np.float32)
    Rk = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    es.es_budget_weighted(ctx, g, big["pi"], torch.as_tensor(v).cuda(), R, True, es.ES_LEARNED_FLOOR, Rk)
    assert np.array_equal(host(Rk), mlp.budget_weighted(big["ref_pi"], cg.din, R, v, True, es.ES_LEARNED_FLOOR))
    # the learned single query equals its stages run one after another
    w = torch.as_tensor(mlp.init_params(5)).cuda()
    es.es_mlp_load(ctx, w)
    vh = torch.empty(g.n, dtype=torch.float32, device="cuda")
    es.es_mlp_infer(ctx, w, F, g.n, c, None, vh)
    es.es_budget_weighted(ctx, g, big["pi"], vh, R, True, es.ES_LEARNED_FLOOR, Rk)
    M = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    es.es_walk_pairs(ctx, g, None, Rk, wl.seed_walk, c, M)
    D = torch.empty(g.n, dtype=torch.float64, device="cuda")
    es.es_diag(ctx, g, Rk, M, c, True, D)
    s_st = torch.empty(g.n, dtype=torch.float64, device="cuda")
    es.es_backward(ctx, g, big["lv"], L, D, c, s_st)
    s_q = torch.empty(g.n, dtype=torch.float64, device="cuda")
    st = es.es_single_source(ctx, g, u, es.make_opts(c, wl.eps, wl.seed_walk, R_SCALE, alloc=es.ES_ALLOC_LEARNED),
                             s_q)
    say(f"learned query: {st.pairs} pairs (stages {int(host(Rk).sum())})")
    assert st.pairs == int(host(Rk).sum())
    assert torch.equal(s_q, s_st)


def test_local_exploitation(es, ctx, big):
    from test_gpu_fullsize import _lde_full
    wl, g, cg, u, L = big["wl"], big["g"], big["cg"], big["u"], big["L"]
    _lde_full(es, ctx, g, cg, u, wl.c, wl.eps, R_SCALE, wl.seed_walk, big["ref_pi"], big["lv"], L)
