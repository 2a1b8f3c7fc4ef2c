"""GPU batches: many sources and uneven graphs in one pass.

A batch must give every source the result of its own single-source query:
identical walk and meeting counts (shared samples, bucketed per source) and
s within float64 summation error; and the oracle's s within 1e-9.  Results may
not depend on the tiling, on hipGraph replay, or on how queries are grouped.
"""
import sys

import numpy as np
import pytest
import torch

import workloads
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


@pytest.fixture(scope="module")
def graphs(es, ctx):
    specs = [(2000,) + workloads.chung_lu(2000, 20000, 11),
             (1 << 15,) + workloads.rmat(1 << 15, 500_000, 5),
             (7000,) + workloads.rmat(7000, 35_000, 8)]
    return [(es.Graph(ctx, n, s, d), OracleGraph(n, s, d)) for n, s, d in specs]


def single(es, ctx, g, u, opts):
    s = torch.empty(g.n, dtype=torch.float64, device="cuda")
    st = es.es_single_source(ctx, g, u, opts, s)
    return s.cpu().numpy(), st


def run_batch(es, ctx, gl, goq, srcs, opts, **kw):
    outs = [torch.full((gl[g].n,), float("nan"), dtype=torch.float64, device="cuda") for g in goq]
    st = es.es_batch(ctx, gl, goq, srcs, opts, outs, **kw)
    return [o.cpu().numpy() for o in outs], st


def pick(og, count, seed):
    return [int(x) for x in workloads.pick_sources(og.n, og.dst, count, seed)]


def test_batch_equals_single_source_and_oracle(es, ctx, graphs):
    g, og = graphs[0]
    srcs = pick(og, 10, 1)
    opts = es.make_opts(C, 1e-4, 31, 1e-3)
    say(f"  batch of {len(srcs)}")
    outs, st = run_batch(es, ctx, [g], [0] * len(srcs), srcs, opts)
    meets = pairs = 0
    for u, s in zip(srcs, outs):
        ref, st1 = single(es, ctx, g, u, opts)
        meets += st1.meets
        pairs += st1.pairs
        assert np.abs(s - ref).max() <= 1e-13
        q = ox.query(og, u, C, 1e-4, 31, 1e-3)
        assert np.abs(s - q["s"]).max() <= 1e-9
    assert st.meets == meets
    assert st.pairs_requested == pairs
    assert st.pairs <= pairs  # shared samples never exceed the per-source total


def test_uneven_multi_graph_batch(es, ctx, graphs):
    gl = [g for g, _ in graphs]
    counts = [3, 70, 9]  # 70 splits into blocks of 64 and 6
    goq, srcs = [], []
    for gi, (cnt, (g, og)) in enumerate(zip(counts, graphs)):
        s = pick(og, cnt, 10 + gi)
        goq += [gi] * cnt
        srcs += s
    # interleave queries so that blocks are gathered by graph, not by position
    order = np.random.default_rng(0).permutation(len(srcs))
    goq = [goq[i] for i in order]
    srcs = [srcs[i] for i in order]
    opts = es.make_opts(C, 1e-6, 5, 1e-7)
    say(f"  uneven batch of {len(srcs)} over {len(gl)} graphs")
    outs, st = run_batch(es, ctx, gl, goq, srcs, opts)
    meets = 0
    for q in range(len(srcs)):
        ref, st1 = single(es, ctx, gl[goq[q]], srcs[q], opts)
        meets += st1.meets
        assert np.abs(outs[q] - ref).max() <= 1e-13, q
    assert st.meets == meets


def test_batch_degenerate_graphs_and_single_source_blocks(es, ctx, graphs):
    """Graphs of one node, without edges, with duplicate edges and self-loops,
    every node a source, next to a one-source block of a larger graph: each
    answer equals its single-source query and the oracle."""
    tiny = [(1, [], []), (3, [], []), (2, [0], [1]), (4, [0, 0, 1], [1, 1, 1])]
    gl, ogs = [], []
    for n, src, dst in tiny:
        gl.append(es.Graph(ctx, n, np.array(src, dtype=np.int32), np.array(dst, dtype=np.int32)))
        ogs.append(OracleGraph(n, src, dst))
    g2, og2 = graphs[2]
    gl.append(g2)
    ogs.append(og2)
    goq, srcs = [], []
    for gi, (n, _, _) in enumerate(tiny):
        goq += [gi] * n
        srcs += list(range(n))
    goq.append(len(tiny))
    srcs.append(pick(og2, 1, 21)[0])
    opts = es.make_opts(C, 1e-3, 3, 1e-3)
    say(f"  batch of {len(srcs)} over {len(gl)} graphs, tiny ones included")
    outs, st = run_batch(es, ctx, gl, goq, srcs, opts, autotune=False)
    meets = 0
    for q, (gi, u) in enumerate(zip(goq, srcs)):
        ref, st1 = single(es, ctx, gl[gi], u, opts)
        meets += st1.meets
        assert np.abs(outs[q] - ref).max() <= 1e-13, (gi, u)
        want = ox.query(ogs[gi], u, C, 1e-3, 3, 1e-3)["s"]
        assert np.abs(outs[q] - want).max() <= 1e-9, (gi, u)
    assert st.meets == meets
    for g in gl[:len(tiny)]:
        g.close()


def test_batch_tilings_agree(es, ctx, graphs):
    g, og = graphs[1]
    srcs = pick(og, 12, 3)
    opts = es.make_opts(C, 1e-6, 7, 1e-7)
    base, st0 = run_batch(es, ctx, [g], [0] * 12, srcs, opts, autotune=False)
    for w in (16, 32, 64):
        for rows in (4, 32, 200):
            say(f"  width={w} rows={rows}")
            outs, st = run_batch(es, ctx, [g], [0] * 12, srcs, opts, autotune=False, force_width=w, force_rows=rows)
            assert st.meets == st0.meets and st.pairs == st0.pairs
            for a, b in zip(base, outs):
                assert np.abs(a - b).max() <= 1e-13


def test_batch_hip_graph_replays(es, ctx, graphs):
    g, og = graphs[2]
    opts = es.make_opts(C, 1e-4, 9, 1e-2)
    for rep, seed in enumerate((1, 2, 3)):
        srcs = pick(og, 8, seed)
        say(f"  replay {rep}")
        eager, st_e = run_batch(es, ctx, [g], [0] * 8, srcs, opts, autotune=False)
        # unrelated eager work between replays
        junk = torch.randn(1 << 20, device="cuda").sum().item()
        assert np.isfinite(junk)
        graph, st_g = run_batch(es, ctx, [g], [0] * 8, srcs, opts, autotune=False, use_hip_graph=True)
        assert st_g.meets == st_e.meets
        for a, b in zip(eager, graph):
            assert np.array_equal(a, b)


def test_batch_long_rows_bitwise_reproducible(es, ctx, graphs):
    """R-MAT 2^15 has in- and out-rows longer than the SpMM's long-row cut
    (1024 entries): their chunk sums are added in chunk order, so eager runs
    and hipGraph replays give the same bits every time."""
    g, og = graphs[1]
    assert og.din.max() > 1024 and og.dout.max() > 1024
    srcs = pick(og, 8, 17)
    opts = es.make_opts(C, 1e-4, 19, 1e-2)
    say(f"  long rows: max in-degree {og.din.max()}, out-degree {og.dout.max()}")
    base, st0 = run_batch(es, ctx, [g], [0] * 8, srcs, opts, autotune=False, force_width=8, force_rows=8)
    for rep in range(4):
        junk = torch.randn(1 << 20, device="cuda").sum().item()
        assert np.isfinite(junk)
        outs, st = run_batch(es, ctx, [g], [0] * 8, srcs, opts, autotune=False, force_width=8, force_rows=8,
                             use_hip_graph=rep > 0)
        assert st.meets == st0.meets
        for a, b in zip(base, outs):
            assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), rep
    for u, s in zip(srcs[:2], base):
        ref, _ = single(es, ctx, g, u, opts)
        assert np.abs(s - ref).max() <= 1e-13


def test_batch_plan_not_reused_for_a_new_graph(es, ctx):
    """Batch on a graph, destroy it, build another graph of the same size and
    batch again with the same sources and options (hipGraph on both times):
    the answer is the new graph's, not a replay of a plan built for the old
    one (whose handle address may be reused)."""
    n = 5000
    srcs = list(range(100, 108))
    opts = es.make_opts(C, 1e-4, 23, 1e-2)
    for rep, seed in enumerate((61, 62, 63)):
        src, dst = workloads.rmat(n, 40_000, seed)
        g = es.Graph(ctx, n, src, dst)
        say(f"  graph {rep} (seed {seed})")
        outs, _ = run_batch(es, ctx, [g], [0] * 8, srcs, opts, autotune=False, use_hip_graph=True)
        og = OracleGraph(n, src, dst)
        for u, s in zip(srcs[:3], outs[:3]):
            ref, _ = single(es, ctx, g, u, opts)
            assert np.abs(s - ref).max() <= 1e-13, (rep, u)
            want = ox.query(og, u, C, 1e-4, 23, 1e-2)["s"]
            assert np.abs(s - want).max() <= 1e-9, (rep, u)
        g.close()


@pytest.mark.parametrize("eps_s", [1e-4, 1e-2])
def test_batch_sparse_levels_equal_single_source(es, ctx, graphs, eps_s):
    """Sparse linearization in a batch: every source keeps the entries its own
    single-source query keeps, so s equals the single-source sparse answer
    (summation order aside) and the oracle's within 1e-9."""
    g, og = graphs[1]
    srcs = pick(og, 10, 4)
    opts = es.make_opts(C, 1e-4, 31, 1e-3, sparse_eps=eps_s)
    outs, st = run_batch(es, ctx, [g], [0] * len(srcs), srcs, opts)
    kept = 0
    for u, s in zip(srcs, outs):
        ref, st1 = single(es, ctx, g, u, opts)
        kept += st1.level_entries
        assert np.abs(s - ref).max() <= 1e-13
    q = ox.query(og, srcs[0], C, 1e-4, 31, 1e-3, sparse_eps=eps_s)
    assert np.abs(outs[0] - q["s"]).max() <= 1e-9
    assert st.level_entries == kept
    assert st.level_bytes == 12 * kept + 8 * g.n * len(srcs)
    say(f"  eps_s={eps_s:g}: {kept} entries kept for {len(srcs)} sources "
        f"({st.level_bytes / 1e6:.1f} MB vs {8 * (st.L + 1) * g.n * len(srcs) / 1e6:.1f} MB dense)")


def test_batch_sparse_uneven_and_hip_graph(es, ctx, graphs):
    """Sparse levels over uneven graphs in one batch, eager and replayed."""
    gl = [graphs[0][0], graphs[2][0]]
    srcs = pick(graphs[0][1], 5, 6) + pick(graphs[2][1], 3, 7)
    goq = [0] * 5 + [1] * 3
    opts = es.make_opts(C, 1e-4, 13, 1e-2, sparse_eps=1e-3)
    eager, st_e = run_batch(es, ctx, gl, goq, srcs, opts, autotune=False)
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda").sum().item()
        assert np.isfinite(junk)
        graph, st_g = run_batch(es, ctx, gl, goq, srcs, opts, autotune=False, use_hip_graph=True)
        assert st_g.level_entries == st_e.level_entries
        for a, b in zip(eager, graph):
            assert np.array_equal(a, b)
    for gi, u, s in zip(goq, srcs, eager):
        ref, _ = single(es, ctx, gl[gi], u, opts)
        assert np.abs(s - ref).max() <= 1e-13


def test_batch_allocation_failure_is_reported_and_recoverable(es, ctx, graphs):
    """A batch whose dense levels cannot be allocated (c = 0.99, eps = 1e-140:
    about 3.2e4 levels of 2^17 x 16 doubles) fails with ES_ENOMEM; the context
    then runs an ordinary batch."""
    n = 1 << 17
    src, dst = workloads.rmat(n, 4 * n, 78)
    g = es.Graph(ctx, n, src, dst)
    srcs = [int(x) for x in workloads.pick_sources(n, dst, 16, 3)]
    L = es.es_num_levels(0.99, 1e-140)
    assert (L + 1) * n * 16 * 8 > 400e9
    bad = es.make_opts(0.99, 1e-140, 1, 1e-290)
    outs = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in srcs]
    with pytest.raises(es.EsError) as e:
        es.es_batch(ctx, [g], [0] * len(srcs), srcs, bad, outs, autotune=False)
    assert e.value.status == es.ES_ENOMEM
    g.close()
    g2, og2 = graphs[2]
    srcs2 = pick(og2, 4, 9)
    opts = es.make_opts(C, 1e-4, 9, 1e-2)
    out2, _ = run_batch(es, ctx, [g2], [0] * 4, srcs2, opts, autotune=False)
    for u, s2 in zip(srcs2, out2):
        ref, _ = single(es, ctx, g2, u, opts)
        assert np.abs(s2 - ref).max() <= 1e-13


def test_batch_autotune_records_choice(es, ctx, graphs):
    g, og = graphs[2]
    srcs = pick(og, 20, 4)
    opts = es.make_opts(C, 1e-4, 9, 1e-3)
    run_batch(es, ctx, [g], [0] * 20, srcs, opts, autotune=True)
    bw = es.es_batch_block_width(g, 20)
    assert bw in (8, 16, 20)
    w, rows = es.es_batch_tuning(g, bw)
    assert w >= bw and w in (8, 16, 32, 64) and rows > 0
    say(f"  20 sources: blocks of {bw}, lane groups of {w}, {rows} entries per lane")


@pytest.mark.parametrize("which", [1, 0])
def test_batch_block_widths_agree(es, ctx, graphs, which):
    """Any source-block width gives every source its single-source answer
    (the same walk and meeting counts; s within float64 summation)."""
    g, og = graphs[which]
    srcs = pick(og, 37, 8)
    opts = es.make_opts(C, 1e-4, 29, 1e-3)
    ref, st0 = run_batch(es, ctx, [g], [0] * 37, srcs, opts, autotune=False)
    for bw in (1, 8, 16, 32, 64):
        outs, st = run_batch(es, ctx, [g], [0] * 37, srcs, opts, autotune=False, block_width=bw)
        assert st.meets == st0.meets and st.pairs_requested == st0.pairs_requested
        for a, b in zip(ref, outs):
            assert np.abs(a - b).max() <= 1e-13, bw
    outs, st = run_batch(es, ctx, [g], [0] * 37, srcs, opts, autotune=True)
    say(f"  graph {which}: autotuned block width {es.es_batch_block_width(g, 37)}")
    for a, b in zip(ref, outs):
        assert np.abs(a - b).max() <= 1e-13
    u, s_ = srcs[5], outs[5]
    single_s, _ = single(es, ctx, g, u, opts)
    assert np.abs(s_ - single_s).max() <= 1e-13


def test_batch_argument_errors(es, ctx, graphs):
    g, og = graphs[0]
    opts = es.make_opts(C, 1e-4, 1, 1e-3)
    out = [torch.empty(g.n, dtype=torch.float64, device="cuda")]
    with pytest.raises(es.EsError):
        es.es_batch(ctx, [g], [1], [0], opts, out)
    with pytest.raises(es.EsError):
        es.es_batch(ctx, [g], [0], [g.n], opts, out)
    with pytest.raises(es.EsError):
        es.es_batch(ctx, [g], [0], [0], opts, out, force_width=12)
    with pytest.raises(es.EsError):
        es.es_batch(ctx, [g], [0], [0], opts, out, block_width=65)
    bad = es.make_opts(C, 1e-4, 1, 1e-3, sparse_eps=1.5)
    with pytest.raises(es.EsError):
        es.es_batch(ctx, [g], [0], [0], bad, out)
