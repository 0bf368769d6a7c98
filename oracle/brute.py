"""Brute-force exact graph quantities from the adjacency matrix (tiny graphs).

TEST INFRASTRUCTURE ONLY. Independent of ``pg_oracle.c``: it never merges
neighbour lists, it multiplies adjacency matrices.

  (A^2)[u, v]  = |N_u cap N_v|
  (A^3)[v, v]  = 2 * (triangles at v)
  trace(A^3)   = 6 * TC
"""
from __future__ import annotations

import numpy as np


def adjacency(g) -> np.ndarray:
    a = np.zeros((g.n, g.n), dtype=np.int64)
    for v in range(g.n):
        for u in g.adj[g.offsets[v]:g.offsets[v + 1]]:
            a[v, int(u)] = 1
    return a


def tc(g) -> int:
    a = adjacency(g)
    t = int(np.trace(a @ a @ a))
    assert t % 6 == 0
    return t // 6


def intersections(g) -> np.ndarray:
    a = adjacency(g)
    return a @ a


def local_cc(g) -> np.ndarray:
    a = adjacency(g)
    d = a.sum(axis=1).astype(np.float64)
    tri2 = np.diag(a @ a @ a).astype(np.float64)
    out = np.zeros(g.n)
    ok = d >= 2
    out[ok] = tri2[ok] / (d[ok] * (d[ok] - 1))
    return out
