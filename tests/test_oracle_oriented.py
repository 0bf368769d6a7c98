"""Pins for the oracle's degree-oriented sets and the oriented triangle count
(Listing "lst:tc"): the sets by their definition on tiny graphs, the exact
oriented sum against adjacency-matrix powers and closed forms, and exactness of
the estimate where a sketch is lossless."""
import math

import numpy as np
import pytest

import oracle
import pggen
from oracle import brute


def _plus_sets_by_definition(g):
    deg = np.diff(g.offsets)
    rank = {v: (int(deg[v]), v) for v in range(g.n)}
    out = []
    for v in range(g.n):
        nb = [int(u) for u in g.adj[g.offsets[v]:g.offsets[v + 1]]]
        out.append(sorted(u for u in nb if rank[u] > rank[v]))
    return out


def _plus_lists(o):
    return [list(map(int, o.adj[o.offsets[v]:o.offsets[v + 1]])) for v in range(o.n)]


def _exact_oriented_sum(g):
    o = oracle.oriented(g)
    eu, ev = oracle.upper_edges(g)
    return int(oracle.exact_pairs(o, eu, ev).astype(np.int64).sum())


def test_oriented_sets_by_definition():
    for bits in range(0, 1 << 10, 7):
        g = pggen.from_adjacency_bits(5, bits)
        assert _plus_lists(oracle.oriented(g)) == _plus_sets_by_definition(g), bits
    for g in (pggen.er(300, 7, seed=2), pggen.rmat(0, 8, seed=3, n=200), pggen.wheel(9), pggen.star(12)):
        o = oracle.oriented(g)
        assert _plus_lists(o) == _plus_sets_by_definition(g)
        eu, _ = oracle.upper_edges(g)
        assert o.nnz == eu.shape[0]  # every undirected edge oriented once
        assert np.array_equal(o.degrees(), np.diff(o.offsets))


def test_oriented_degree_bound():
    # in degree order every d+_v is at most sqrt(2 m)
    for g in (pggen.rmat(12, 16, seed=1), pggen.er(2000, 30, seed=4), pggen.complete(50)):
        m = g.nnz // 2
        assert int(oracle.oriented(g).degrees().max()) <= math.isqrt(2 * m)


def test_exact_oriented_sum_is_the_triangle_count():
    for bits in range(1 << 10):
        g = pggen.from_adjacency_bits(5, bits)
        assert _exact_oriented_sum(g) == brute.tc(g), bits
    for n in (3, 6, 11):
        assert _exact_oriented_sum(pggen.complete(n)) == math.comb(n, 3)
    assert _exact_oriented_sum(pggen.wheel(8)) == 8
    assert _exact_oriented_sum(pggen.friendship(6)) == 6
    assert _exact_oriented_sum(pggen.complete_bipartite(4, 6)) == 0
    for seed in (1, 2):
        g = pggen.er(120, 9, seed=seed)
        assert _exact_oriented_sum(g) == brute.tc(g)


def test_onehash_oriented_tc_exact_when_k_covers_the_unions():
    """1-hash with k >= |N+_u cup N+_v| for every edge (k = 2 max d+) is exact
    (Section 4.4), so the oriented estimate is the exact triangle count."""
    g = pggen.rmat(10, 16, seed=2)
    o = oracle.oriented(g)
    k = 2 * int(o.degrees().max())
    sk = oracle.build_sketches(o, oracle.KIND_1H, k, 1, seed=4)
    assert oracle.tc_oriented(g, sk, "1h") == float(oracle.exact_tc(g))


def test_bf_oriented_tc_exact_when_hashes_are_injective():
    """With b = 1 and a hash that maps all n IDs to distinct bits, the AND of
    two filters has exactly |N+_u cap N+_v| ones, so the L estimator (c / b) is
    the exact triangle count (Section 4.2)."""
    g = pggen.er(300, 10, seed=6)
    B = 1 << 20
    for seed in range(1, 200):  # a seed whose bit index is injective on V
        a, c = oracle.hash_consts(oracle.KIND_BF, seed, 1)
        if len({oracle.bf_index(int(a[0]), int(c[0]), x, B) for x in range(g.n)}) == g.n:
            break
    else:
        raise AssertionError("no injective seed found")
    sk = oracle.build_sketches(oracle.oriented(g), oracle.KIND_BF, B, 1, seed)
    assert oracle.tc_oriented(g, sk, "l") == float(oracle.exact_tc(g))


def test_kh_oriented_tc_zero_on_triangle_free_graphs():
    # disjoint oriented sets give no positional matches (Section 4.3)
    for g in (pggen.complete_bipartite(5, 9), pggen.cycle(12), pggen.star(30)):
        sk = oracle.build_sketches(oracle.oriented(g), oracle.KIND_KH, 16, 1, seed=2)
        assert oracle.tc_oriented(g, sk, "kh") == 0.0
