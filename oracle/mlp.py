"""Budget network of the learned allocation, float64 reference (test infrastructure).

The sample budget of Section 3.2 follows from the variance bound of Lemma 1,
Var[s^L(j)] <= 1/((1-sqrt c)^4 R) sum_k pi_i(k)^2 pi_j(k)^2 D(k,k)(1 - D(k,k)) / rho(k)
(the proof keeps the Bernoulli variance D(1-D) before bounding it by 1).
Minimising the worst case over j of that sum under a fixed total gives
rho(k) proportional to pi_i(k)^2 D(k,k)(1-D(k,k)); the paper drops the
variance factor.  The learned allocation keeps it, with the meeting
probability p(k) = 1 - D(k,k) predicted by a small network from local degree
features, v(k) = p(k)(1-p(k)), and

    R(k) = ceil( (R * pi(k)^2) * (w(k) / wbar) ),  w(k) = max(v(k), f * vbar),
    vbar = (sum_k Q(pi(k)^2 v(k))) / (sum_k Q(pi(k)^2)),  Q(x) = round(x * 2^62),
    wbar likewise with w,

sums over nodes that take samples, in exact integer arithmetic, so the total
stays that of the pi^2 rule.  The floor f (default 1/2) keeps every node at
no less than about f times its pi^2 share (see budget_weighted).  The prediction only moves samples between nodes:
every node with pi(k) > 0 still gets at least one pair (v is floored at
V_FLOOR), so D^ stays unbiased whatever the network says.

Network: 6 features -> 64 -> 64 -> 1 (ReLU), p = c * sigmoid(z), since two
walks meet at all only if both take step 1 (probability c).  D(k,k) is a
property of the graph around v_k alone (Algorithm 2 starts both walks at
v_k whatever the query), so every feature is source-independent and one
prediction per node serves every query on the graph.  Loss: the
R-weighted binomial cross-entropy of p against the observed meeting fraction
M(k)/R(k), weights capped.

Parameter layout (4673 floats): W1 [64][6], b1 [64], W2 [64][64], b2 [64],
w3 [64], b3 [1].
"""
from __future__ import annotations

import math

import numpy as np

NF, H = 6, 64
NPARAM = H * NF + H + H * H + H + H + 1
V_FLOOR = 1e-6
WEIGHT_CAP = 65536
FLOOR_RATIO = 0.5


def labels(R, M):
    """Observed meeting fraction y = M/R and loss weight w = min(R, cap)."""
    R = np.asarray(R, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    y = np.where(R > 0, M / np.maximum(R, 1), 0.0)
    w = np.minimum(R, WEIGHT_CAP)
    return y, w


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    o = 0
    W1 = theta[o:o + H * NF].reshape(H, NF); o += H * NF
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    w3 = theta[o:o + H]; o += H
    b3 = theta[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, [b3]])


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases (float32 values, as the GPU stores them)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W1 = rng.uniform(-1, 1, (H, NF)) * math.sqrt(6.0 / NF)
    W2 = rng.uniform(-1, 1, (H, H)) * math.sqrt(6.0 / H)
    w3 = rng.uniform(-1, 1, H) * math.sqrt(6.0 / H)
    return pack(W1, np.zeros(H), W2, np.zeros(H), w3, 0.0).astype(np.float32)


def features(g, c: float) -> np.ndarray:
    """Per node: log1p d_in, log1p d_out, log1p mean and log1p max in-degree of
    the in-neighbours, the mean over in-neighbours a of 1/d_in(a) (0 for
    d_in(a) = 0), and c/d_in (the exact probability that two walks meet at
    step 1, Lemma 4 with l = 1).  Rows of nodes without in-neighbours carry
    zeros in columns 2-5."""
    n = g.n
    din = g.din.astype(np.float64)
    dout = g.dout.astype(np.float64)
    F = np.zeros((n, NF))
    F[:, 0] = np.log1p(din)
    F[:, 1] = np.log1p(dout)
    nb_din = din[g.in_idx]  # in-degree of every in-neighbour, rows of the in-CSR
    row = np.repeat(np.arange(n), g.din)
    sums = np.bincount(row, weights=nb_din, minlength=n)
    maxs = np.zeros(n)
    np.maximum.at(maxs, row, nb_din)
    recip = np.where(nb_din > 0, 1.0 / np.maximum(nb_din, 1.0), 0.0)
    rsums = np.bincount(row, weights=recip, minlength=n)
    has = g.din > 0
    F[:, 2] = np.log1p(np.where(has, sums / np.maximum(din, 1), 0.0))
    F[:, 3] = np.log1p(np.where(has, maxs, 0.0))
    F[:, 4] = np.where(has, rsums / np.maximum(din, 1), 0.0)
    F[:, 5] = np.where(has, c / np.maximum(din, 1), 0.0)
    return F


def features_at(g, c: float, nodes) -> np.ndarray:
    """The rows of `features` for the given nodes only, one node at a time
    (for graphs too large to form every row on the CPU)."""
    nodes = np.asarray(nodes, dtype=np.int64)
    F = np.zeros((len(nodes), NF))
    for r, k in enumerate(nodes):
        d = int(g.din[k])
        nb = g.in_idx[g.in_off[k]:g.in_off[k + 1]]
        nb_din = g.din[nb].astype(np.float64)
        F[r, 0] = math.log1p(d)
        F[r, 1] = math.log1p(float(g.dout[k]))
        if d > 0:
            F[r, 2] = math.log1p(nb_din.sum() / d)
            F[r, 3] = math.log1p(nb_din.max())
            F[r, 4] = sum(1.0 / x for x in nb_din if x > 0) / d
            F[r, 5] = c / d
    return F


def forward(theta, X, c):
    """Return (p, cache) for inputs X [N][6]."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ w3 + b3
    sig = 1.0 / (1.0 + np.exp(-z))
    p = c * sig
    return p, (X, a1, h1, a2, h2, z)


def loss(theta, X, y, w, c) -> float:
    p, _ = forward(theta, X, c)
    bce = -(y * np.log(p) + (1 - y) * np.log1p(-p))
    return float(np.sum(w * bce) / np.sum(w))


def grad(theta, X, y, w, c):
    """Analytic gradient of `loss` by the chain rule, layer by layer."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    p, (X, a1, h1, a2, h2, z) = forward(theta, X, c)
    Wt = np.sum(w)
    # dL/dp = w/Wt * (-y/p + (1-y)/(1-p)), dp/dz = p (1 - p/c)
    gz = (w / Wt) * (1.0 - p / c) * (-y + (1.0 - y) * p / (1.0 - p))
    dw3 = h2.T @ gz
    db3 = np.sum(gz)
    da2 = np.outer(gz, w3) * (a2 > 0)
    dW2 = da2.T @ h1
    db2 = da2.sum(0)
    da1 = (da2 @ W2) * (a1 > 0)
    dW1 = da1.T @ X
    db1 = da1.sum(0)
    return pack(dW1, db1, dW2, db2, dw3, db3)


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def predict_variance(theta, X, c) -> np.ndarray:
    p, _ = forward(theta, X, c)
    return np.maximum(p * (1 - p), V_FLOOR)


def budget_weighted(pi, din, R, v, exact_small_din=True, floor_ratio=FLOOR_RATIO) -> np.ndarray:
    """R(k) = ceil((R * (pi*pi)) * (w(k) * (S2 / S3))) over the nodes that
    take samples, with exact fixed-point sums

        S1 = sum Q(pi^2 v),  S2 = sum Q(pi^2),  vbar = S1 / S2,
        w(k) = max(v(k), floor_ratio * vbar),  S3 = sum Q(pi^2 w).

    The floor keeps every node within a fixed factor of its pi^2 share:
    Bernstein's inequality, behind the error guarantee of Theorem 1, has a
    range term besides the variance, and a node left with very few pairs
    has a heavy-tailed error even when its variance is small.  floor_ratio
    = 0 gives w = v."""
    v = np.asarray(v, dtype=np.float32).astype(np.float64)
    p2 = pi * pi
    take = pi > 0
    if exact_small_din:
        take &= din >= 2
    q1 = np.rint((p2 * v) * 2.0 ** 62).astype(np.int64)
    q2 = np.rint(p2 * 2.0 ** 62).astype(np.int64)
    S1 = int(q1[take].sum())
    S2 = int(q2[take].sum())
    thr = floor_ratio * (float(S1) / float(S2)) if S1 > 0 else 0.0
    w = np.maximum(v, thr)
    q3 = np.rint((p2 * w) * 2.0 ** 62).astype(np.int64)
    S3 = int(q3[take].sum())
    want = R * p2
    if S3 > 0:
        want = want * (w * (float(S2) / float(S3)))
    Rk = np.ceil(want)
    Rk[~take] = 0.0
    return Rk.astype(np.uint64)
