"""Training data and training of the learned walk budget.

Labels come from the method itself: Algorithm 2 (`es_walk_pairs`) run with a
uniform number of pairs on every node of a training graph estimates each
node's meeting probability 1 - D(k,k); features come from `es_mlp_features`.
Training runs on the GPU with the library's own gradient and Adam kernels
(`es_mlp_train`).
Device buffers are PyTorch tensors; every computation is a library call.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import binding as es

NPARAM = 4673


def init_weights(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases; layout W1[64][6], b1, W2[64][64], b2, w3, b3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W1 = rng.uniform(-1, 1, (64, 6)) * math.sqrt(6.0 / 6)
    W2 = rng.uniform(-1, 1, (64, 64)) * math.sqrt(6.0 / 64)
    w3 = rng.uniform(-1, 1, 64) * math.sqrt(6.0 / 64)
    return np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), w3, [0.0]]).astype(np.float32)


def collect(ctx: es.Context, g: es.Graph, c: float, pairs_per_node: int, seed: int):
    """(features [n][6] float32, R, M uint64) for every node of g, on the device."""
    F = torch.empty((g.n, 6), dtype=torch.float32, device="cuda")
    es.es_mlp_features(ctx, g, c, F)
    R = torch.full((g.n,), pairs_per_node, dtype=torch.uint64, device="cuda")
    M = torch.empty(g.n, dtype=torch.uint64, device="cuda")
    es.es_walk_pairs(ctx, g, None, R, seed, c, M)
    return F, R, M


def train(ctx: es.Context, F, R, M, c: float, epochs: int = 400, lr: float = 3e-3, seed: int = 7):
    """Train from scratch; returns (weights tensor on the device, losses per epoch)."""
    w = torch.as_tensor(init_weights(seed)).cuda()
    losses = es.es_mlp_train(ctx, F, R, M, F.shape[0], c, epochs, lr, w)
    return w, losses
