"""Seeded synthetic graph generators: shape, set semantics, reproducibility."""
import numpy as np
import pytest

import workloads


@pytest.mark.parametrize("gen,n,m", [("rmat", 1 << 14, 200_000), ("rmat", 10_000, 80_000),
                                      ("chung_lu", 2000, 20000), ("chung_lu", 50_000, 300_000)])
def test_generator_is_a_set_without_loops(gen, n, m):
    src, dst = getattr(workloads, gen)(n, m, 7)
    assert len(src) == m and len(dst) == m
    assert src.min() >= 0 and dst.min() >= 0 and src.max() < n and dst.max() < n
    assert not np.any(src == dst)
    key = src.astype(np.int64) * n + dst
    assert np.all(np.diff(key) > 0)  # sorted and distinct


def test_generator_reproducible_and_seeded():
    a = workloads.rmat(1 << 12, 30000, 5)
    b = workloads.rmat(1 << 12, 30000, 5)
    c = workloads.rmat(1 << 12, 30000, 6)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert not np.array_equal(a[1], c[1])


def test_power_law_shape():
    src, dst = workloads.rmat(1 << 16, 1_000_000, 3)
    din = np.bincount(dst, minlength=1 << 16)
    assert din.max() > 50 * din.mean()
    src, dst = workloads.chung_lu(20000, 200_000, 3)
    dout = np.bincount(src, minlength=20000)
    assert dout[0] == dout.max()  # node 0 is the largest hub


def test_sources_have_two_in_neighbours():
    src, dst = workloads.rmat(1 << 14, 100_000, 9)
    s = workloads.pick_sources(1 << 14, dst, 8, 1)
    din = np.bincount(dst, minlength=1 << 14)
    assert len(set(s.tolist())) == 8 and np.all(din[s] >= 2)


def test_uneven_parts():
    parts = workloads.uneven_parts()
    assert len(parts) == 12
    assert parts[0].n == 10_000 and parts[-1].n == 2_000_000
    counts = workloads.uneven_source_counts(12, 256, 42)
    assert counts.sum() == 256 and counts.min() >= 1 and counts.max() > 4 * counts.min()
