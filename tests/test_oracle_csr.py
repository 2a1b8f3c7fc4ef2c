"""The CSR oracle passes (C loops for billion-edge graphs) against the
sparse-matrix oracle: same in-neighbour lists, forward levels bit for bit,
back-accumulation to rounding."""
import numpy as np
import pytest

import workloads
from graphs import complete, cycle, hub_graph, random_graph, siblings, three_sources
from oracle import csr
from oracle import exactsim as ox
from oracle.graph import OracleGraph

C = 0.6

GRAPHS = {
    "chung_lu_2k": lambda: (2000,) + workloads.chung_lu(2000, 20000, 11),
    "rmat_32k": lambda: (1 << 15,) + workloads.rmat(1 << 15, 500_000, 5),
    "hubs": lambda: hub_graph(30000, 20000, 20000, 60000, 3),
    "cycle": lambda: cycle(1000),
    "complete5": lambda: complete(5),
    "random_small": lambda: random_graph(50, 200, 1),
    "three_sources": lambda: three_sources(),
    "siblings": lambda: siblings(),
}


def pair(name):
    n, src, dst = GRAPHS[name]()
    og = OracleGraph(n, src, dst)
    return og, csr.CsrGraph(n, og.src, og.dst)


@pytest.mark.parametrize("name", list(GRAPHS))
def test_csr_graph_matches_sparse_oracle(name):
    og, cg = pair(name)
    assert cg.m == og.m
    assert np.array_equal(cg.din, og.din)
    assert np.array_equal(cg.dout, og.dout)
    assert np.array_equal(cg.inv_din.view(np.uint64), og.inv_din.view(np.uint64))
    assert np.array_equal(cg.in_off, og.in_off)
    assert np.array_equal(cg.in_idx, og.in_idx)


@pytest.mark.parametrize("name", list(GRAPHS))
def test_forward_bitwise_and_backward(name):
    og, cg = pair(name)
    rng = np.random.default_rng(3)
    for u in sorted({0, og.n - 1, int(np.argmax(og.din))}):
        for eps in (1e-2, 1e-6):
            L = ox.num_levels(C, eps)
            ref_lv, ref_pi = ox.forward_levels(og, u, C, L)
            lv, pi = csr.forward_levels(cg, u, C, L)
            assert np.array_equal(lv.view(np.uint64), ref_lv.view(np.uint64))
            assert np.array_equal(pi.view(np.uint64), ref_pi.view(np.uint64))
            D = rng.uniform(1 - C, 1, og.n)
            ref_s = ox.back_accumulate(og, ref_lv, D, C)
            s = csr.back_accumulate(cg, lv, D, C)
            assert np.abs(s - ref_s).max() <= 1e-15 * max(1.0, np.abs(ref_s).max())


@pytest.mark.parametrize("bad", ["unsorted", "duplicate", "self_loop", "range"])
def test_rejects_malformed_edge_lists(bad):
    src = np.array([0, 0, 1, 2], dtype=np.int32)
    dst = np.array([1, 2, 2, 0], dtype=np.int32)
    if bad == "unsorted":
        src, dst = src[::-1].copy(), dst[::-1].copy()
    elif bad == "duplicate":
        src[1], dst[1] = 0, 1
    elif bad == "self_loop":
        dst[2] = 1
    else:
        dst[3] = 7
    with pytest.raises(ValueError):
        csr.CsrGraph(3, src, dst)


@pytest.mark.parametrize("name", ["chung_lu_2k", "rmat_32k", "three_sources"])
def test_features_one_node_at_a_time(name):
    from oracle import mlp
    og, cg = pair(name)
    ref = mlp.features(og, C)
    nodes = np.unique(np.concatenate([np.arange(min(og.n, 50)), np.random.default_rng(2).integers(0, og.n, 200)]))
    for g in (og, cg):
        got = mlp.features_at(g, C, nodes)
        assert np.allclose(got, ref[nodes], rtol=1e-14, atol=1e-15)
