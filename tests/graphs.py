"""Small hand-built graphs shared by the tests (edge lists only)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name: str) -> float:
    with open(os.path.join(GOLDEN, "closed_forms.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, val = line.split()[:2]
            if key == name:
                return float(val)
    raise KeyError(name)


def complete(n):
    s, d = zip(*[(i, j) for i in range(n) for j in range(n) if i != j])
    return n, np.array(s), np.array(d)


def cycle(n):
    s = np.arange(n)
    return n, s, (s + 1) % n


def siblings():
    # 0 -> 1, 0 -> 2: nodes 1 and 2 share their only in-neighbour
    return 3, np.array([0, 0]), np.array([1, 2])


def three_sources():
    # 1, 2, 3 (no in-neighbours) -> 0
    return 4, np.array([1, 2, 3]), np.array([0, 0, 0])


def random_graph(n, m, seed):
    rng = np.random.default_rng(seed)
    s = rng.integers(0, n, m)
    d = rng.integers(0, n, m)
    return n, s, d


def hub_graph(n, hub_in, hub_out, extra, seed):
    """A random graph plus one node with `hub_in` in-neighbours and one with
    `hub_out` out-neighbours (long CSR rows in both directions)."""
    rng = np.random.default_rng(seed)
    s = [rng.integers(0, n, extra)]
    d = [rng.integers(0, n, extra)]
    s.append(rng.choice(n, hub_in, replace=False))
    d.append(np.full(hub_in, 1))
    s.append(np.full(hub_out, 2))
    d.append(rng.choice(n, hub_out, replace=False))
    return n, np.concatenate(s), np.concatenate(d)


def diamond():
    # 1 -> 0, 2 -> 0, 3 -> 1, 3 -> 2, 4 -> 3, 0 -> 4: two paths from 0 reach 3
    return 5, np.array([1, 2, 3, 3, 4, 0]), np.array([0, 0, 1, 2, 3, 4])


def fork():
    # 2 -> 1, 3 -> 1, 1 -> 0, 4 -> 0: nodes 2, 3, 4 have no in-neighbours
    return 5, np.array([2, 3, 1, 4]), np.array([1, 1, 0, 0])


def lde_rounds():
    """{graph name: (node, [edges counted per round])} from lde_rounds.txt."""
    out = {}
    with open(os.path.join(GOLDEN, "lde_rounds.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            parts = line.split()
            out[parts[0]] = (int(parts[1]), [int(x) for x in parts[2:]])
    return out
