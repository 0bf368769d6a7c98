"""Pins for the oracle's exact quantities: closed forms and brute force."""
import math

import numpy as np
import pytest

import oracle
import pggen
from oracle import brute


def _edge_intersections(g):
    eu, ev = oracle.upper_edges(g)
    return eu, ev, oracle.exact_pairs(g, eu, ev)


@pytest.mark.parametrize("n", [3, 4, 5, 8, 17, 40])
def test_complete_graph(n):
    g = pggen.complete(n)
    eu, ev, inter = _edge_intersections(g)
    assert eu.shape[0] == n * (n - 1) // 2
    assert np.all(inter == n - 2)
    assert oracle.exact_tc(g) == math.comb(n, 3) == oracle.exact_tc_listing(g)
    assert np.allclose(oracle.exact_cc(g), 1.0)
    assert np.allclose(oracle.exact_jaccard(g, eu, ev), (n - 2) / n)


@pytest.mark.parametrize("leaves", [1, 2, 10])
def test_star(leaves):
    g = pggen.star(leaves)
    _, _, inter = _edge_intersections(g)
    assert np.all(inter == 0)
    assert oracle.exact_tc(g) == 0 == oracle.exact_tc_listing(g)
    assert np.all(oracle.exact_cc(g) == 0)
    if leaves >= 2:
        # two leaves share exactly the hub
        assert oracle.exact_pairs(g, [1], [2])[0] == 1
        assert oracle.exact_jaccard(g, [1], [2])[0] == 1.0


@pytest.mark.parametrize("n,tc", [(3, 1), (4, 0), (5, 0), (12, 0)])
def test_cycle(n, tc):
    g = pggen.cycle(n)
    assert oracle.exact_tc(g) == tc == oracle.exact_tc_listing(g)


@pytest.mark.parametrize("rim", [4, 5, 9])
def test_wheel(rim):
    g = pggen.wheel(rim)
    assert oracle.exact_tc(g) == rim == oracle.exact_tc_listing(g)
    cc = oracle.exact_cc(g)
    assert cc[0] == pytest.approx(2.0 / (rim - 1))
    assert np.allclose(cc[1:], 2.0 / 3.0)


@pytest.mark.parametrize("a,b", [(1, 1), (2, 5), (4, 4)])
def test_complete_bipartite(a, b):
    g = pggen.complete_bipartite(a, b)
    _, _, inter = _edge_intersections(g)
    assert np.all(inter == 0) and oracle.exact_tc(g) == 0
    if a >= 2:
        # two vertices on the same side have identical neighbourhoods
        assert oracle.exact_pairs(g, [0], [1])[0] == b


@pytest.mark.parametrize("k", [1, 3, 7])
def test_friendship(k):
    g = pggen.friendship(k)
    assert oracle.exact_tc(g) == k == oracle.exact_tc_listing(g)


def test_empty_and_isolated():
    g = pggen.from_pairs(5, [], [])
    assert oracle.upper_edges(g)[0].shape[0] == 0
    assert oracle.exact_tc(g) == 0 == oracle.exact_tc_listing(g)
    assert np.all(oracle.exact_cc(g) == 0)
    assert oracle.exact_jaccard(g, [0], [1])[0] == 0.0


def _against_brute(g):
    a2 = brute.intersections(g)
    eu, ev, inter = _edge_intersections(g)
    assert np.array_equal(inter, a2[eu, ev])
    t = brute.tc(g)
    assert oracle.exact_tc(g) == t == oracle.exact_tc_listing(g)
    assert np.allclose(oracle.exact_cc(g), brute.local_cc(g), rtol=0, atol=1e-15)
    # non-adjacent pairs too
    rng = np.random.default_rng(g.n)
    u = rng.integers(0, g.n, 20)
    v = rng.integers(0, g.n, 20)
    assert np.array_equal(oracle.exact_pairs(g, u, v), a2[u, v])


def test_every_graph_on_five_vertices():
    for bits in range(1 << 10):
        _against_brute(pggen.from_adjacency_bits(5, bits))


def test_every_graph_on_six_vertices_sampled():
    rng = np.random.default_rng(6)
    for bits in rng.choice(1 << 15, size=2000, replace=False):
        _against_brute(pggen.from_adjacency_bits(6, int(bits)))


@pytest.mark.parametrize("seed", range(6))
def test_random_graphs_against_brute(seed):
    _against_brute(pggen.er(40 + 10 * seed, 6 + seed, seed=seed))
    _against_brute(pggen.rmat(0, 8, seed=seed, n=60))


def test_disjoint_union_adds():
    parts = [pggen.complete(6), pggen.wheel(5), pggen.friendship(3), pggen.cycle(3)]
    g = pggen.disjoint_union(*parts)
    assert oracle.exact_tc(g) == sum(oracle.exact_tc(p) for p in parts) == 20 + 5 + 3 + 1
