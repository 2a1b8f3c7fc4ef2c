"""GPU sparse linearization (Section 3.2, Lemma 2) against the oracle: the
kept entries of every level bit for bit, whole queries with the sampled,
the exact and the Algorithm 3 diagonals, the stored-entry statistics, and
the edge cases (tiny graphs, a coarse threshold, L = 0, a list too
small for the entries, invalid arguments)."""
import math
import sys

import numpy as np
import pytest
import torch

import workloads
from graphs import cycle, hub_graph, random_graph
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
    "cycle_40": lambda: cycle(40),
}
_cache = {}


def pair(es, ctx, name):
    if name not in _cache:
        n, s, d = GRAPHS[name]()
        say(f"[graph {name}]")
        _cache[name] = (es.Graph(ctx, n, s, d), OracleGraph(n, s, d))
    return _cache[name]


def gpu_sparse_levels(es, ctx, g, u, L, eps_s):
    cap = es.es_sparse_capacity(g.n, g.m, L, C, eps_s)
    idx = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
    val = torch.empty(max(cap, 1), dtype=torch.float64, device="cuda")
    pi = torch.empty(g.n, dtype=torch.float64, device="cuda")
    counts = es.es_forward_sparse(ctx, g, u, C, L, eps_s, idx, val, pi)
    return counts, host(idx), host(val), pi


def check_levels(counts, idx, val, ref_lv, theta):
    """Level l of the list holds exactly the oracle's entries > theta, bit for bit."""
    pos = 0
    for l in range(ref_lv.shape[0]):
        want = np.flatnonzero(ref_lv[l] > theta)
        assert counts[l] == len(want), l
        got_i = idx[pos:pos + counts[l]]
        got_v = val[pos:pos + counts[l]]
        order = np.argsort(got_i)
        assert np.array_equal(got_i[order], want), l
        assert np.array_equal(got_v[order].view(np.uint64), ref_lv[l][want].view(np.uint64)), l
        pos += counts[l]
    return pos


@pytest.mark.parametrize("name", ["chung_lu_2k", "rmat_32k", "hubs", "cycle_40"])
@pytest.mark.parametrize("eps_s", [1e-2, 1e-4, 1e-6])
def test_kept_entries_bitwise(es, ctx, name, eps_s):
    g, og = pair(es, ctx, name)
    u = int(np.argmax(og.din)) if name != "cycle_40" else 7
    L = ox.num_levels(C, 1e-6)
    counts, idx, val, pi = gpu_sparse_levels(es, ctx, g, u, L, eps_s)
    ref_lv, ref_pi = ox.forward_levels(og, u, C, L)
    theta = ox.sparse_threshold(C, eps_s)
    kept = check_levels(counts, idx, val, ref_lv, theta)
    assert kept <= 1.0 / theta
    # the full pi is the dense forward pass's, bit for bit
    assert np.array_equal(host(pi).view(np.uint64), ref_pi.view(np.uint64))
    say(f"  {name} eps_s={eps_s:g}: {kept} of {(L + 1) * g.n} entries kept")


def test_list_too_small(es, ctx):
    g, og = pair(es, ctx, "chung_lu_2k")
    L = 10
    ref_lv, _ = ox.forward_levels(og, 0, C, L)
    theta = ox.sparse_threshold(C, 1e-3)
    need = int(np.count_nonzero(ref_lv > theta))
    idx = torch.empty(need - 1, dtype=torch.int32, device="cuda")
    val = torch.empty(need - 1, dtype=torch.float64, device="cuda")
    with pytest.raises(es.EsError) as e:
        es.es_forward_sparse(ctx, g, 0, C, L, 1e-3, idx, val)
    assert e.value.args[0].endswith(f"(status {es.ES_EOVERFLOW})")
    # exactly enough room succeeds
    idx = torch.empty(need, dtype=torch.int32, device="cuda")
    val = torch.empty(need, dtype=torch.float64, device="cuda")
    counts = es.es_forward_sparse(ctx, g, 0, C, L, 1e-3, idx, val)
    assert sum(counts) == need


@pytest.mark.parametrize("name", ["chung_lu_2k", "rmat_32k", "hubs"])
def test_single_source_against_oracle(es, ctx, name):
    g, og = pair(es, ctx, name)
    u = int(np.argmax(og.din))
    eps, r_scale, seed = 1e-4, 1e-3, 21
    s = torch.empty(g.n, dtype=torch.float64, device="cuda")
    s_dense = torch.empty(g.n, dtype=torch.float64, device="cuda")
    st_d = es.es_single_source(ctx, g, u, es.make_opts(C, eps, seed, r_scale), s_dense)
    for eps_s in (eps, 1e-2):
        st = es.es_single_source(ctx, g, u, es.make_opts(C, eps, seed, r_scale, sparse_eps=eps_s), s)
        ref = ox.query(og, u, C, eps, seed, r_scale, sparse_eps=eps_s)
        err = np.abs(host(s) - ref["s"]).max()
        kept = int(np.count_nonzero(ref["kept"]))
        diff = host(s_dense) - host(s)
        say(f"  {name} eps_s={eps_s:g}: max|s - oracle| {err:.1e}, {kept} entries kept "
            f"({st.level_bytes / 1e6:.2f} MB vs {st_d.level_bytes / 1e6:.2f} MB dense), "
            f"dense - sparse in [{diff.min():.1e}, {diff.max():.1e}]")
        assert err <= S_TOL
        # the walks are those of the dense query
        assert st.pairs == st_d.pairs and st.meets == st_d.meets
        assert st.level_entries == kept
        assert st.level_bytes == 12 * kept + 8 * g.n
        assert st.workspace_bytes >= st.level_bytes
        assert st_d.level_entries == (st_d.L + 1) * g.n
        # Lemma 2: the removed entries lower s by at most eps_s (D^ is in [0, 1])
        assert diff.min() >= -1e-12 and diff.max() <= eps_s


def test_exact_diagonal_against_power_method(es, ctx):
    """With the exact diagonal the sparse query stays within c^(L+1) + eps_s
    of the Power Method."""
    g, og = pair(es, ctx, "chung_lu_2k")
    S = sr.power_method(og, C, 60)
    D = sr.exact_diagonal(og, S, C)
    Dd = torch.as_tensor(D).cuda()
    s = torch.empty(g.n, dtype=torch.float64, device="cuda")
    eps = 1e-4
    L = ox.num_levels(C, eps)
    for eps_s in (1e-4, 1e-3):
        for u in (0, 5, 300):
            es.es_single_source(ctx, g, u, es.make_opts(C, eps, 1, 1.0, d_override=Dd, sparse_eps=eps_s), s)
            ref = ox.query(og, u, C, eps, 1, d_override=D, sparse_eps=eps_s)
            assert np.abs(host(s) - ref["s"]).max() <= S_TOL
            assert sr.max_error(host(s), S[:, u]) <= C ** (L + 1) + eps_s


@pytest.mark.parametrize("mode", [1, 2])
def test_with_local_exploitation(es, ctx, mode):
    """Algorithm 3 with sparse levels: the plan reads only the graph and R(k),
    the back-accumulation the kept entries (one dense working slot)."""
    g, og = pair(es, ctx, "rmat_32k")
    u = int(np.argmax(og.din))
    eps, r_scale, seed, eps_s = 1e-4, 1e-3, 77, 1e-4
    s = torch.empty(g.n, dtype=torch.float64, device="cuda")
    st = es.es_single_source(ctx, g, u, es.make_opts(C, eps, seed, r_scale, lde=mode, sparse_eps=eps_s), s)
    L = ox.num_levels(C, eps)
    lv, pi = ox.forward_levels(og, u, C, L)
    Rk = ox.budget(pi, og.din, ox.total_samples(og.n, C, eps, r_scale), True)
    ell, z, R2 = lde.plan(og, Rk, C, mode)
    M = ox.walk_counts(og, R2, seed, C, nonstop=ell)
    D = lde.diag_estimate(R2, M, ell, z, C, og.din)
    kept = ox.sparsify_levels(lv, ox.sparse_threshold(C, eps_s))
    ref = ox.back_accumulate(og, kept, D, C)
    err = np.abs(host(s) - ref).max()
    say(f"  mode {mode}: l(u)={st.lde_source_level} max|s - oracle| {err:.1e}")
    assert err <= S_TOL
    assert st.pairs == int(R2.sum())
    assert st.level_bytes == 12 * int(np.count_nonzero(kept)) + 8 * g.n


def test_tiny_graphs(es, ctx):
    """Empty and tiny graphs, sources without in-neighbours, a coarse
    threshold, L = 2, and L = 0 (level 0 alone)."""
    cases = [(1, [], []), (3, [], []), (2, [0], [1]), (4, [0, 0, 1], [1, 1, 1]),
             (5, [1, 2, 3, 4, 2, 3], [0, 0, 0, 0, 1, 1]), (6, [0, 1, 2, 3, 4, 5], [1, 2, 3, 4, 5, 0])]
    sc = math.sqrt(C)
    coarse = 0.999  # theta = 0.05: level 1 keeps pi^1(i) = sqrt(c)(1 - sqrt c)/d_in(u) only for d_in(u) <= 3
    for n, src, dst in cases:
        g = es.Graph(ctx, n, np.array(src, dtype=np.int32), np.array(dst, dtype=np.int32))
        og = OracleGraph(n, src, dst)
        s = torch.empty(n, dtype=torch.float64, device="cuda")
        for u in range(n):
            for eps in (1e-3, 0.9):
                for eps_s in (1e-3, coarse):
                    for mode in (0, 2):
                        es.es_single_source(ctx, g, u, es.make_opts(C, eps, 3, 1e-2, lde=mode, sparse_eps=eps_s), s)
                        L = ox.num_levels(C, eps)
                        lv, pi = ox.forward_levels(og, u, C, L)
                        Rk = ox.budget(pi, og.din, ox.total_samples(n, C, eps, 1e-2), True)
                        if mode:
                            ell, z, R2 = lde.plan(og, Rk, C, mode)
                            M = ox.walk_counts(og, R2, 3, C, nonstop=ell)
                            D = lde.diag_estimate(R2, M, ell, z, C, og.din)
                        else:
                            M = ox.walk_counts(og, Rk, 3, C)
                            D = ox.diag_estimate(Rk, M, og.din, C)
                        kept = ox.sparsify_levels(lv, ox.sparse_threshold(C, eps_s))
                        ref = ox.back_accumulate(og, kept, D, C)
                        assert np.abs(host(s) - ref).max() <= S_TOL, (n, u, eps, eps_s, mode)
        # L = 0: level 0 alone
        counts, idx, val, _ = gpu_sparse_levels(es, ctx, g, 0, 0, 1e-3)
        assert counts == [1] and idx[0] == 0 and val[0] == 1 - sc


def test_sparse_argument_errors(es, ctx):
    g, og = pair(es, ctx, "random_small")
    s = torch.empty(g.n, dtype=torch.float64, device="cuda")
    for bad in (-1e-3, 1.0, 2.0, float("nan")):
        with pytest.raises(es.EsError) as e:
            es.es_single_source(ctx, g, 0, es.make_opts(C, 1e-3, 1, 1e-2, sparse_eps=bad), s)
        assert e.value.args[0].endswith(f"(status {es.ES_EINVAL})")
    idx = torch.empty(16, dtype=torch.int32, device="cuda")
    val = torch.empty(16, dtype=torch.float64, device="cuda")
    for bad in (0.0, -1.0, 1.0):
        with pytest.raises(es.EsError):
            es.es_forward_sparse(ctx, g, 0, C, 5, bad, idx, val)
    with pytest.raises(es.EsError):
        es.es_forward_sparse(ctx, g, g.n, C, 5, 1e-3, idx, val)
    with pytest.raises(es.EsError):
        es.es_sparse_capacity(10, 10, 5, C, 0.0)
    # batches check the option too
    sb = torch.empty(g.n, dtype=torch.float64, device="cuda")
    with pytest.raises(es.EsError) as e:
        es.es_batch(ctx, [g], [0], [0], es.make_opts(C, 1e-3, 1, 1e-2, sparse_eps=-1.0), [sb])
    assert e.value.args[0].endswith(f"(status {es.ES_EINVAL})")
