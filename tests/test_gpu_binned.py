"""GPU parity of the binned (push-form) level pass against the oracle and
the pull pass: pi^l bit for bit, the back-accumulation within 1e-12 and
repeatable bit for bit, whole queries (dense and sparse linearization) within
the query tolerance.  The graphs cover one bin and several, a ragged last bin,
push lists longer than a scatter range and bins longer than an accumulate item
(split into partial sums), nodes without in- or out-neighbours."""
import sys

import numpy as np
import pytest
import torch

import workloads
from graphs import cycle, hub_graph, random_graph, three_sources
from oracle import exactsim as ox
from oracle.graph import OracleGraph

pytestmark = pytest.mark.gpu

C = 0.6


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


def host(t):
    return t.cpu().numpy()


GRAPHS = {
    "three_sources": lambda: three_sources(),
    "cycle_1000": lambda: cycle(1000),
    "random_5000": lambda: random_graph(5000, 40000, 3),
    "chung_lu_20001": lambda: (20001,) + workloads.chung_lu(20001, 200000, 12),
    "rmat_32k": lambda: (1 << 15,) + workloads.rmat(1 << 15, 500_000, 5),
    # a node with 1.1e6 in-neighbours and one with 1.1e6 out-neighbours: push
    # lists cut over several scatter ranges, bins split over several items
    "hubs_1e6": lambda: hub_graph(1_200_000, 1_100_000, 1_100_000, 400_000, 4),
}

_cache = {}


def pair(es, ctx, name):
    if name not in _cache:
        n, src, dst = GRAPHS[name]()
        say(f"[graph {name}] n={n} m={len(src)}")
        base = es.ES_DEDUP | es.ES_DROP_SELF_LOOPS
        gb = es.Graph(ctx, n, src, dst, base | es.ES_LEVELS_BINNED)
        gp = es.Graph(ctx, n, src, dst, base | es.ES_LEVELS_PULL)
        assert gb.binned and not gp.binned
        _cache[name] = (gb, gp, OracleGraph(n, src, dst))
    return _cache[name]


def forward(es, ctx, g, u, L):
    lv = torch.empty((L + 1) * g.n, dtype=torch.float64, device="cuda")
    pi = torch.empty(g.n, dtype=torch.float64, device="cuda")
    es.es_forward(ctx, g, u, C, L, lv, pi)
    return lv, pi


@pytest.mark.parametrize("name", list(GRAPHS))
def test_binned_forward_bitwise(es, ctx, name):
    gb, gp, og = pair(es, ctx, name)
    for u in sorted({0, og.n - 1, int(np.argmax(og.din)), int(np.argmax(og.dout))}):
        L = ox.num_levels(C, 1e-6)
        say(f"  forward u={u} L={L}")
        lv, pi = forward(es, ctx, gb, u, L)
        ref_lv, ref_pi = ox.forward_levels(og, u, C, L)
        assert np.array_equal(host(lv).reshape(L + 1, og.n).view(np.uint64), ref_lv.view(np.uint64))
        assert np.array_equal(host(pi).view(np.uint64), ref_pi.view(np.uint64))
        lvp, _ = forward(es, ctx, gp, u, L)
        assert torch.equal(lv, lvp)


@pytest.mark.parametrize("name", list(GRAPHS))
def test_binned_backward(es, ctx, name):
    gb, gp, og = pair(es, ctx, name)
    u = int(np.argmax(og.din))
    L = ox.num_levels(C, 1e-6)
    D = np.random.default_rng(7).uniform(1 - C, 1.0, og.n)
    Dt = dev(D, torch.float64)
    lv, _ = forward(es, ctx, gb, u, L)
    outs = []
    for g in (gb, gb, gp):
        s = torch.empty(og.n, dtype=torch.float64, device="cuda")
        es.es_backward(ctx, g, lv, L, Dt, C, s)
        outs.append(host(s))
    ref_lv, _ = ox.forward_levels(og, u, C, L)
    ref = ox.back_accumulate(og, ref_lv, D, C)
    say(f"  backward: max|binned - oracle| = {np.abs(outs[0] - ref).max():.3g}, "
        f"max|binned - pull| = {np.abs(outs[0] - outs[2]).max():.3g}")
    assert np.abs(outs[0] - ref).max() <= 1e-12
    assert np.abs(outs[0] - outs[2]).max() <= 1e-13
    assert np.array_equal(outs[0].view(np.uint64), outs[1].view(np.uint64))


@pytest.mark.parametrize("name,r_scale,sparse_eps", [("random_5000", 1e-4, 0.0), ("chung_lu_20001", 1e-4, 0.0),
                                                     ("chung_lu_20001", 1e-4, 1e-3), ("hubs_1e6", 1e-6, 1e-4)])
def test_binned_query(es, ctx, name, r_scale, sparse_eps):
    gb, gp, og = pair(es, ctx, name)
    u = int(np.argmax(og.din))
    eps = 1e-4
    opts = es.make_opts(C, eps, 9, r_scale, sparse_eps=sparse_eps)
    sb = torch.empty(og.n, dtype=torch.float64, device="cuda")
    sp = torch.empty(og.n, dtype=torch.float64, device="cuda")
    stb = es.es_single_source(ctx, gb, u, opts, sb)
    stp = es.es_single_source(ctx, gp, u, opts, sp)
    say(f"  query: {stb.pairs} pairs")
    assert stb.pairs == stp.pairs and stb.meets == stp.meets
    ref = ox.query(og, u, C, eps, 9, r_scale, sparse_eps=sparse_eps)
    assert stb.meets == int(ref["M"].sum())
    err = np.abs(host(sb) - ref["s"]).max()
    say(f"  query sparse_eps={sparse_eps}: max|binned - oracle| = {err:.3g}")
    assert err <= 1e-9
    assert np.abs(host(sb) - host(sp)).max() <= 1e-13


def test_level_pass_flags(es, ctx):
    n, src, dst = random_graph(100, 400, 2)
    g = es.Graph(ctx, n, src, dst)
    assert not g.binned  # small graphs take the pull pass by default
    for flags in (es.ES_LEVELS_PULL | es.ES_LEVELS_BINNED, 16, 1 << 31):
        with pytest.raises(es.EsError) as e:
            es.Graph(ctx, n, src, dst, flags)
        assert e.value.status == es.ES_EINVAL
    # one node, no edges: one bin, no scatter range
    g1 = es.Graph(ctx, 1, np.array([], np.int32), np.array([], np.int32), es.ES_LEVELS_BINNED)
    lv, pi = forward(es, ctx, g1, 0, 3)
    ref_lv, ref_pi = ox.forward_levels(OracleGraph(1, [], []), 0, C, 3)
    assert np.array_equal(host(lv).view(np.uint64), ref_lv.reshape(-1).view(np.uint64))
    s = torch.empty(1, dtype=torch.float64, device="cuda")
    es.es_single_source(ctx, g1, 0, es.make_opts(C, 1e-3, 1, 1e-3), s)
    assert host(s)[0] == 1.0
