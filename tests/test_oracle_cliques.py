"""Pins for the oracle's 4-clique counts (Listing "lst:fcl"): brute force over
every 4-subset of small graphs, closed forms, additivity over disjoint unions,
and for the Bloom-filter estimate the one-sided error of membership queries and
exactness when the hash is injective on the vertex IDs."""
import itertools
import math

import numpy as np
import pytest

import oracle
import pggen
from oracle import brute


def _brute_four_cliques(g):
    a = brute.adjacency(g) > 0
    cnt = 0
    for q in itertools.combinations(range(g.n), 4):
        if all(a[x, y] for x, y in itertools.combinations(q, 2)):
            cnt += 1
    return cnt


def test_every_graph_on_five_vertices():
    for bits in range(1 << 10):
        g = pggen.from_adjacency_bits(5, bits)
        assert oracle.four_cliques(g) == _brute_four_cliques(g), bits


def test_graphs_on_six_vertices_sampled():
    rng = np.random.default_rng(6)
    for bits in rng.integers(0, 1 << 15, 600):
        g = pggen.from_adjacency_bits(6, int(bits))
        assert oracle.four_cliques(g) == _brute_four_cliques(g), int(bits)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_graphs_against_brute_force(seed):
    g = pggen.er(28, 12, seed=seed)
    assert oracle.four_cliques(g) == _brute_four_cliques(g)


def test_closed_forms():
    for n in (3, 4, 5, 9, 20):
        assert oracle.four_cliques(pggen.complete(n)) == math.comb(n, 4)
    assert oracle.four_cliques(pggen.complete_bipartite(6, 7)) == 0
    assert oracle.four_cliques(pggen.wheel(3)) == 1  # the wheel on a triangle is K4
    assert oracle.four_cliques(pggen.wheel(8)) == 0
    assert oracle.four_cliques(pggen.friendship(5)) == 0
    # complete tripartite K_{2,2,2} (octahedron): largest clique is a triangle
    s, d = [], []
    for x in range(6):
        for y in range(x + 1, 6):
            if x // 2 != y // 2:
                s.append(x)
                d.append(y)
    assert oracle.four_cliques(pggen.from_pairs(6, s, d)) == 0


def test_disjoint_union_adds():
    parts = [pggen.complete(7), pggen.wheel(3), pggen.er(60, 10, seed=4), pggen.complete(5)]
    g = pggen.disjoint_union(*parts)
    assert oracle.four_cliques(g) == sum(oracle.four_cliques(p) for p in parts)


def test_bf_estimate_never_below_exact():
    for g, B, b in ((pggen.rmat(10, 16, seed=2), 128, 1), (pggen.er(500, 20, seed=1), 256, 2),
                    (pggen.complete(30), 64, 1)):
        sk = oracle.build_sketches(oracle.oriented(g), oracle.KIND_BF, B, b, seed=3)
        assert oracle.four_cliques_bf(g, sk) >= oracle.four_cliques(g)


def test_bf_estimate_exact_when_hashes_are_injective():
    g = pggen.er(200, 24, seed=2)
    B = 1 << 20
    for seed in range(1, 200):
        a, c = oracle.hash_consts(oracle.KIND_BF, seed, 1)
        if len({oracle.bf_index(int(a[0]), int(c[0]), x, B) for x in range(g.n)}) == g.n:
            break
    else:
        raise AssertionError("no injective seed found")
    sk = oracle.build_sketches(oracle.oriented(g), oracle.KIND_BF, B, 1, seed)
    exact = oracle.four_cliques(g)
    assert exact > 0 and oracle.four_cliques_bf(g, sk) == exact
