"""Pins of the float64 budget network and the weighted allocation (CPU)."""
import math

import numpy as np
import pytest
import torch

from graphs import three_sources
from oracle import exactsim as ox
from oracle import mlp
from oracle.graph import OracleGraph

C = 0.6


def data(seed, N=300):
    rng = np.random.default_rng(seed)
    theta = mlp.init_params(seed).astype(np.float64)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(theta)
    theta = mlp.pack(W1, rng.normal(0, 0.3, 64), W2, rng.normal(0, 0.3, 64), w3, -1.0)
    X = rng.normal(0, 1, (N, 6))
    R = rng.integers(0, 5000, N)
    M = (R * rng.uniform(0, C, N)).astype(np.int64)
    y, w = mlp.labels(R, M)
    return theta, X, y, w


def test_gradient_matches_central_differences():
    theta, X, y, w = data(1)
    g = mlp.grad(theta, X, y, w, C)
    rng = np.random.default_rng(0)
    idx = np.concatenate([rng.choice(mlp.NPARAM, 60, replace=False), [mlp.NPARAM - 1, 0, 384]])
    h = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (mlp.loss(tp, X, y, w, C) - mlp.loss(tm, X, y, w, C)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * (1 + abs(g[i])), (i, fd, g[i])


def test_gradient_matches_autograd():
    theta, X, y, w = data(2)
    t = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    o = 0
    W1 = t[o:o + 384].view(64, 6); o += 384
    b1 = t[o:o + 64]; o += 64
    W2 = t[o:o + 4096].view(64, 64); o += 4096
    b2 = t[o:o + 64]; o += 64
    w3 = t[o:o + 64]; o += 64
    b3 = t[o]
    Xt = torch.tensor(X)
    p = C * torch.sigmoid(torch.relu(torch.relu(Xt @ W1.T + b1) @ W2.T + b2) @ w3 + b3)
    yt, wt = torch.tensor(y), torch.tensor(w)
    L = (wt * -(yt * torch.log(p) + (1 - yt) * torch.log1p(-p))).sum() / wt.sum()
    L.backward()
    assert abs(L.item() - mlp.loss(theta, X, y, w, C)) < 1e-12
    assert np.abs(t.grad.numpy() - mlp.grad(theta, X, y, w, C)).max() < 1e-12


def test_adam_constant_gradient_closed_form():
    theta = np.zeros(5)
    g = np.array([0.5, -2.0, 1e-3, 3.0, -0.1])
    m = np.zeros(5)
    v = np.zeros(5)
    for t in range(1, 6):
        prev = theta.copy()
        theta, m, v = mlp.adam_step(theta, g, m, v, t, 0.01)
        # bias-corrected moments equal g and g^2, so each step is lr * g / (|g| + eps)
        assert np.allclose(prev - theta, 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_features_on_hand_built_graph():
    n, s, d = three_sources()
    g = OracleGraph(n, s, d)
    F = mlp.features(g, C)
    # node 0: three in-neighbours, none of which has an in-neighbour
    assert F[0].tolist() == pytest.approx([math.log1p(3), 0.0, 0.0, 0.0, 0.0, C / 3])
    assert F[1].tolist() == pytest.approx([0.0, math.log1p(1), 0.0, 0.0, 0.0, 0.0])
    # 0 -> 1, 2 -> 1, 3 -> 2, 4 -> 2, 5 -> 2: I(1) = {0, 2}, d_in(0) = 0, d_in(2) = 3
    g = OracleGraph(6, [0, 2, 3, 4, 5], [1, 1, 2, 2, 2])
    F = mlp.features(g, C)
    assert F[1].tolist() == pytest.approx([math.log1p(2), 0.0, math.log1p(1.5), math.log1p(3), 1 / 6, C / 2])
    assert F[2].tolist() == pytest.approx([math.log1p(3), math.log1p(1), 0.0, 0.0, 0.0, C / 3])
    assert F[3].tolist() == pytest.approx([0.0, math.log1p(1), 0.0, 0.0, 0.0, 0.0])


def test_labels():
    y, w = mlp.labels([0, 10, 100000], [0, 3, 50000])
    assert y.tolist() == [0.0, 0.3, 0.5]
    assert w.tolist() == [0.0, 10.0, mlp.WEIGHT_CAP]


def test_weighted_budget_properties():
    rng = np.random.default_rng(4)
    n = 5000
    pi = rng.random(n) ** 6
    pi[rng.random(n) < 0.2] = 0.0
    pi /= pi.sum()  # a PPR vector: sum <= 1 keeps the fixed-point sums below 2^63
    din = rng.integers(0, 30, n)
    R = 1e12
    base = ox.budget(pi, din, R)
    v1 = np.full(n, 0.2, dtype=np.float32)
    r1 = mlp.budget_weighted(pi, din, R, v1, floor_ratio=0.0)
    # constant v reproduces the pi^2 rule up to the rounding of v / vbar
    assert np.abs(r1.astype(np.int64) - base.astype(np.int64)).max() <= 1
    v = rng.uniform(1e-4, 0.25, n).astype(np.float32)
    r = mlp.budget_weighted(pi, din, R, v, floor_ratio=0.0)
    take = (pi > 0) & (din >= 2)
    assert np.all(r[take] >= 1) and np.all(r[~take] == 0)
    # the total stays that of the pi^2 rule (ceil adds at most one per node)
    assert abs(int(r.sum()) - int(base.sum())) <= take.sum()
    # doubling v changes nothing but rounding
    r2 = mlp.budget_weighted(pi, din, R, 2 * v, floor_ratio=0.0)
    assert np.abs(r2.astype(np.int64) - r.astype(np.int64)).max() <= 1
    # nodes with larger predicted variance get more samples per unit of pi^2
    k = np.argsort(-pi * take)[:50]
    ratio = r[k] / (R * pi[k] ** 2)
    assert np.corrcoef(ratio, v[k])[0, 1] > 0.99


def test_weighted_budget_floor():
    rng = np.random.default_rng(6)
    n = 5000
    pi = rng.random(n) ** 6
    pi[rng.random(n) < 0.2] = 0.0
    pi /= pi.sum()
    din = rng.integers(0, 30, n)
    R = 1e12
    take = (pi > 0) & (din >= 2)
    v = (10.0 ** rng.uniform(-6, np.log10(0.25), n)).astype(np.float32)
    base = ox.budget(pi, din, R)
    p2 = pi * pi
    vbar = (p2[take] * v[take]).sum() / p2[take].sum()
    for f in (0.0, 0.125, 0.5, 1.0):
        r = mlp.budget_weighted(pi, din, R, v, floor_ratio=f)
        assert np.all(r[take] >= 1) and np.all(r[~take] == 0)
        assert abs(int(r.sum()) - int(base.sum())) <= take.sum()
        w = np.maximum(v.astype(np.float64), f * vbar)
        wbar = (p2[take] * w[take]).sum() / p2[take].sum()
        # every node keeps at least f * vbar / wbar of its pi^2 share
        assert np.all(r[take] >= np.floor(f * vbar / wbar * R * p2[take] * (1 - 1e-12)))
        # above the floor the weights stay proportional to v
        k = np.argsort(-pi * take * (v >= f * vbar))[:50]
        assert np.corrcoef(r[k] / (R * p2[k]), v[k])[0, 1] > 0.99
    # a floor of one raises every node to at least vbar
    r1 = mlp.budget_weighted(pi, din, R, v, floor_ratio=1.0)
    small = take & (v < 0.01 * vbar) & (R * p2 > 1e4)
    assert small.sum() > 10
    assert np.all(r1[small] >= 0.5 * base[small])


def test_variance_weighting_beats_pi2_with_exact_variance():
    # the allocation itself: with the exact meeting probabilities in place of
    # the network, the weighted budget reduces the error at equal pairs
    import workloads
    from oracle import simrank as sr
    src, dst = workloads.chung_lu(600, 5000, 21)
    g = OracleGraph(600, src, dst)
    S = sr.power_method(g, C, 60)
    D = sr.exact_diagonal(g, S, C)
    v = np.maximum((1 - D) * D, mlp.V_FLOOR)
    eps = 1e-3
    L = ox.num_levels(C, eps)
    lv, pi = ox.forward_levels(g, 0, C, L)
    R = ox.total_samples(g.n, C, eps, 1e-3)
    e_pi2, e_v = [], []
    for seed in range(4):
        for rule, errs in ((ox.budget(pi, g.din, R), e_pi2),
                           (mlp.budget_weighted(pi, g.din, R, v, floor_ratio=0.0), e_v)):
            M = ox.walk_counts(g, rule, 50 + seed, C)
            s = ox.back_accumulate(g, lv, ox.diag_estimate(rule, M, g.din, C), C)
            errs.append(np.abs(s - S[:, 0]).max())
    assert np.mean(e_v) < np.mean(e_pi2)
