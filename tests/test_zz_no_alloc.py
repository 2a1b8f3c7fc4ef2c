"""The allocation-free top-k entry point (es_topk_noalloc) against es_topk.

Two calls in a row, the second on a smaller input (fewer nodes, smaller k),
each equal to es_topk on the same scores; the device's free memory does not
change across the allocation-free calls once the library is loaded.
"""
import ctypes
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def free_bytes():
    hip = ctypes.CDLL("libamdhip64.so")
    free, total = ctypes.c_size_t(), ctypes.c_size_t()
    assert hip.hipMemGetInfo(ctypes.byref(free), ctypes.byref(total)) == 0
    return free.value


def scores(n, seed):
    # coarse values: ties everywhere, including at the k-th score
    rng = np.random.default_rng(seed)
    return torch.as_tensor(rng.integers(0, 64, n) / 64.0).cuda()


def test_topk_noalloc_matches_topk_twice():
    from paper_2004_03493_amd import binding as es
    ctx = es.Context(0)
    cases = [(200_000, 4096, 17, 1), (3_000, 500, -1, 2)]  # second call: smaller n and k
    outs = []
    for n, k, excl, seed in cases:
        s = scores(n, seed)
        idx = torch.empty(k, dtype=torch.int32, device="cuda")
        val = torch.empty(k, dtype=torch.float64, device="cuda")
        outs.append((n, k, excl, s, idx, val))
    # load the library's kernels once (module loading may allocate)
    es.es_topk_noalloc(ctx, outs[1][3], outs[1][0], -1, 1, outs[1][4])
    torch.cuda.synchronize()
    before = free_bytes()
    for n, k, excl, s, idx, val in outs:
        say(f"  noalloc n={n} k={k} exclude={excl}")
        es.es_topk_noalloc(ctx, s, n, excl, k, idx, val)
    torch.cuda.synchronize()
    after = free_bytes()
    assert after == before, (before, after)
    for n, k, excl, s, idx, val in outs:
        ref_i = torch.empty(k, dtype=torch.int32, device="cuda")
        ref_v = torch.empty(k, dtype=torch.float64, device="cuda")
        es.es_topk(ctx, s, n, excl, k, ref_i, ref_v)
        assert torch.equal(idx, ref_i) and torch.equal(val, ref_v)
        # and against a host sort by (score desc, id asc)
        h = s.cpu().numpy()
        order = np.lexsort((np.arange(n), -h))
        order = order[order != excl][:k]
        assert np.array_equal(idx.cpu().numpy(), order)
    # sizes beyond the fixed scratch are refused
    big = torch.empty(5000, dtype=torch.int32, device="cuda")
    with pytest.raises(es.EsError) as e:
        es.es_topk_noalloc(ctx, outs[0][3], outs[0][0], -1, 5000, big)
    assert e.value.status == es.ES_EINVAL
    ctx.close()
