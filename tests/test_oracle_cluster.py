"""Pins for the oracle's vertex similarities (Listing "lst:sim"), Jarvis-Patrick
clustering (Listing "lst:cl") and cluster labels: closed forms on named graphs,
set arithmetic by brute force, reachability by adjacency-matrix powers and
scipy's connected components."""
import itertools

import numpy as np
import pytest

import oracle
import pggen
from oracle import brute

CN, JAC, OVL, TOT = oracle.SIM_COMMON, oracle.SIM_JACCARD, oracle.SIM_OVERLAP, oracle.SIM_TOTAL


def _sets(g):
    return [set(int(x) for x in g.adj[g.offsets[v]:g.offsets[v + 1]]) for v in range(g.n)]


# ---- similarity -------------------------------------------------------------------------

@pytest.mark.parametrize("n", [3, 4, 7, 12])
def test_similarity_complete_graph(n):
    g = pggen.complete(n)
    eu, ev = oracle.upper_edges(g)
    assert np.all(oracle.exact_similarity(g, eu, ev, CN) == n - 2)
    assert np.allclose(oracle.exact_similarity(g, eu, ev, JAC), (n - 2) / n)
    assert np.allclose(oracle.exact_similarity(g, eu, ev, OVL), (n - 2) / (n - 1))
    assert np.all(oracle.exact_similarity(g, eu, ev, TOT) == n)


@pytest.mark.parametrize("a,b", [(2, 3), (4, 4), (3, 7)])
def test_similarity_complete_bipartite(a, b):
    g = pggen.complete_bipartite(a, b)
    # two vertices of the first side share the whole second side
    u = np.array([0] * (a - 1), np.int32)
    v = np.arange(1, a, dtype=np.int32)
    assert np.all(oracle.exact_similarity(g, u, v, CN) == b)
    assert np.all(oracle.exact_similarity(g, u, v, JAC) == 1.0)
    assert np.all(oracle.exact_similarity(g, u, v, OVL) == 1.0)
    assert np.all(oracle.exact_similarity(g, u, v, TOT) == b)
    # across the sides nothing is shared and the union is everything
    eu, ev = oracle.upper_edges(g)
    for m in (CN, JAC, OVL):
        assert np.all(oracle.exact_similarity(g, eu, ev, m) == 0.0)
    assert np.all(oracle.exact_similarity(g, eu, ev, TOT) == a + b)


def test_similarity_star_and_isolated():
    g = pggen.disjoint_union(pggen.star(6), pggen.from_pairs(2, [], []))
    # leaves 1 and 2 share only the hub; the two isolated vertices 7, 8 share nothing
    u, v = np.array([1, 7, 0], np.int32), np.array([2, 8, 7], np.int32)
    assert list(oracle.exact_similarity(g, u, v, CN)) == [1, 0, 0]
    assert list(oracle.exact_similarity(g, u, v, JAC)) == [1.0, 0.0, 0.0]
    assert list(oracle.exact_similarity(g, u, v, OVL)) == [1.0, 0.0, 0.0]
    assert list(oracle.exact_similarity(g, u, v, TOT)) == [1, 0, 6]


def test_similarity_against_set_arithmetic():
    """Every pair of every graph on five vertices: the measures from Python set
    operations on the neighbour lists (no merge, no formula for the union)."""
    pairs = np.array(list(itertools.combinations(range(5), 2)), np.int32)
    for bits in range(0, 1 << 10, 3):
        g = pggen.from_adjacency_bits(5, bits)
        nb = _sets(g)
        want = {CN: [], JAC: [], OVL: [], TOT: []}
        for u, v in pairs:
            a, b = nb[u], nb[v]
            want[CN].append(len(a & b))
            want[JAC].append(len(a & b) / len(a | b) if a | b else 0.0)
            want[OVL].append(len(a & b) / min(len(a), len(b)) if a and b else 0.0)
            want[TOT].append(len(a | b))
        for m, w in want.items():
            got = oracle.exact_similarity(g, pairs[:, 0], pairs[:, 1], m)
            assert np.allclose(got, w, rtol=0, atol=1e-15), (bits, m)


def test_similarity_clamps_estimates():
    du, dv = np.array([4, 4, 4, 0]), np.array([6, 6, 6, 3])
    est = np.array([-1.0, 2.5, 9.0, 0.7])
    assert list(oracle.similarity_from_intersection(du, dv, est, CN)) == list(est)
    assert np.allclose(oracle.similarity_from_intersection(du, dv, est, OVL), [0.0, 2.5 / 4, 1.0, 0.0])
    assert np.allclose(oracle.similarity_from_intersection(du, dv, est, TOT), [10.0, 7.5, 6.0, 3.0])
    assert np.allclose(oracle.similarity_from_intersection(du, dv, est, JAC), [0.0, 2.5 / 7.5, 4 / 6, 0.0])


def test_similarity_onehash_exact_when_k_covers_degrees():
    """1-hash with k at least |N_u cup N_v| estimates the intersection exactly
    (Section 4.4: the union's bottom-k is the whole union), so with k = 2 d_max
    every similarity equals the exact one."""
    g = pggen.er(300, 6, seed=5)
    k = 2 * int(g.degrees().max())
    sk = oracle.build_sketches(g, oracle.KIND_1H, k, 1, seed=3)
    eu, ev = oracle.upper_edges(g)
    for m in (CN, JAC, OVL, TOT):
        assert np.allclose(oracle.similarity(sk, "1h", eu, ev, m), oracle.exact_similarity(g, eu, ev, m),
                           rtol=1e-12, atol=1e-12)


# ---- Jarvis-Patrick -----------------------------------------------------------------------

def _two_cliques_and_bridge():
    a, b = np.triu_indices(5, 1)
    src = np.concatenate([a, a + 5, [4]])
    dst = np.concatenate([b, b + 5, [5]])
    return pggen.from_pairs(10, src, dst)


def test_jarvis_patrick_two_cliques():
    g = _two_cliques_and_bridge()
    eu, ev = oracle.upper_edges(g)
    bridge = (eu == 4) & (ev == 5)
    for m, tau in ((CN, 0.5), (JAC, 0.0), (OVL, 0.0)):
        keep = oracle.exact_jarvis_patrick(g, m, tau)
        assert keep.dtype == np.uint8
        assert keep[bridge].tolist() == [0] and np.all(keep[~bridge] == 1)
        lab = oracle.clusters(g.n, eu, ev, keep)
        assert lab.tolist() == [0] * 5 + [5] * 5
        assert oracle.cluster_count(lab) == 2
    # every edge of the graph: one cluster
    assert oracle.cluster_count(oracle.clusters(g.n, eu, ev)) == 1


@pytest.mark.parametrize("k", [1, 3, 6])
def test_jarvis_patrick_threshold_is_strict(k):
    g = pggen.friendship(k)  # every edge has exactly one common neighbour
    eu, ev = oracle.upper_edges(g)
    assert np.all(oracle.exact_jarvis_patrick(g, CN, 0.999) == 1)
    none = oracle.exact_jarvis_patrick(g, CN, 1.0)
    assert np.all(none == 0)
    assert oracle.clusters(g.n, eu, ev, none).tolist() == list(range(g.n))


def test_jarvis_patrick_cycle_keeps_nothing():
    g = pggen.cycle(9)
    assert np.all(oracle.exact_jarvis_patrick(g, CN, 0.0) == 0)
    assert np.all(oracle.exact_jarvis_patrick(g, TOT, 3.5) == 1)  # |N_u cup N_v| = 4 on every edge


# ---- cluster labels -----------------------------------------------------------------------

def _reachability_labels(g):
    a = brute.adjacency(g) > 0
    r = np.eye(g.n, dtype=bool) | a
    for _ in range(g.n):
        r = r | ((r.astype(np.int64) @ a.astype(np.int64)) > 0)
    return np.array([int(np.flatnonzero(r[v])[0]) for v in range(g.n)])


def test_clusters_every_graph_on_five_vertices():
    for bits in range(1 << 10):
        g = pggen.from_adjacency_bits(5, bits)
        eu, ev = oracle.upper_edges(g)
        assert oracle.clusters(g.n, eu, ev).tolist() == _reachability_labels(g).tolist(), bits


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_clusters_against_scipy(seed):
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    g = pggen.er(3000, 1.5, seed=seed)
    eu, ev = oracle.upper_edges(g)
    keep = (np.random.default_rng(seed).random(eu.shape[0]) < 0.7).astype(np.uint8)
    lab = oracle.clusters(g.n, eu, ev, keep)
    sel = keep.astype(bool)
    a = coo_matrix((np.ones(int(sel.sum())), (eu[sel], ev[sel])), shape=(g.n, g.n))
    ncomp, comp = connected_components(a, directed=False)
    assert oracle.cluster_count(lab) == ncomp
    # same partition, each part labelled by its smallest vertex
    first = np.full(ncomp, g.n, np.int64)
    np.minimum.at(first, comp, np.arange(g.n))
    assert np.array_equal(lab, first[comp])


def test_clusters_long_path_and_empty():
    n = 200
    v = np.arange(n - 1)
    perm = np.random.default_rng(7).permutation(n)
    g = pggen.from_pairs(n, perm[v], perm[v + 1])  # one path through the vertices in random order
    eu, ev = oracle.upper_edges(g)
    assert np.all(oracle.clusters(n, eu, ev) == 0)
    assert oracle.clusters(n, eu, ev, np.zeros(eu.shape[0], np.uint8)).tolist() == list(range(n))
    assert oracle.clusters(0, np.zeros(0, np.int32), np.zeros(0, np.int32)).shape == (0,)


def test_clusters_disjoint_union_blocks():
    parts = [pggen.complete(4), pggen.cycle(5), pggen.star(3), pggen.wheel(4)]
    g = pggen.disjoint_union(*parts)
    eu, ev = oracle.upper_edges(g)
    lab = oracle.clusters(g.n, eu, ev)
    starts = np.cumsum([0] + [p.n for p in parts[:-1]])
    want = np.repeat(starts, [p.n for p in parts])
    assert np.array_equal(lab, want) and oracle.cluster_count(lab) == len(parts)
