"""Pins for the oracle's 4-clique counts (Listing "lst:fcl"): brute force over
every 4-subset of small graphs, closed forms, additivity over disjoint unions,
for the Bloom-filter membership estimate its one-sided error and exactness when
the hash is injective on the vertex IDs, and for the estimate from the AND (or
OR) of the filter of N+_w and a filter of C3 a brute-force transcription of the
definition, one (edge, w) per triangle, and the limit estimator's exactness
under injective hashes."""
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


# ---- sketch intersections: filter of N+_w AND filter of C3 ---------------------

def _injective_seed(n, B, b):
    """A seed whose b hash functions put the n vertex IDs on b * n distinct bits."""
    for seed in range(1, 400):
        a, c = oracle.hash_consts(oracle.KIND_BF, seed, b)
        bits = {oracle.bf_index(int(a[h]), int(c[h]), x, B) for x in range(n) for h in range(b)}
        if len(bits) == b * n:
            return seed
    raise AssertionError("no injective seed found")


def _brute_filter_counts(g, sk):
    """Histograms of c (AND) and c_or (OR) and the size sum, straight from the
    definitions with Python sets: C3 per oriented edge, its filter from the
    hash helper, each w in C3 against the filter row of N+_w."""
    o = oracle.oriented(g)
    plus = [set(o.adj[o.offsets[v]:o.offsets[v + 1]].tolist()) for v in range(g.n)]
    B, b = sk.size, sk.b
    a, c = oracle.hash_consts(oracle.KIND_BF, sk.seed, b)
    ha = np.zeros(B + 1, np.uint64)
    ho = np.zeros(B + 1, np.uint64)
    sizes = 0
    for u in range(g.n):
        for v in plus[u]:
            c3 = plus[u] & plus[v]
            fbits = {oracle.bf_index(int(a[h]), int(c[h]), x, B) for x in c3 for h in range(b)}
            for w in c3:
                row = sk.words[w]
                wbits = {t for t in range(B) if (int(row[t >> 6]) >> (t & 63)) & 1}
                ha[len(wbits & fbits)] += 1
                ho[len(wbits | fbits)] += 1
                sizes += len(plus[w]) + len(c3)
    return ha, ho, sizes


@pytest.mark.parametrize("case", ["er28", "k9", "wheel3", "rmat7"])
def test_filter_counts_against_brute_force(case):
    g = {"er28": lambda: pggen.er(28, 12, seed=5), "k9": lambda: pggen.complete(9),
         "wheel3": lambda: pggen.wheel(3), "rmat7": lambda: pggen.rmat(7, 8, seed=2)}[case]()
    for B, b in ((64, 1), (192, 2)):
        sk = oracle.build_sketches(oracle.oriented(g), oracle.KIND_BF, B, b, seed=6)
        ha, ho, sizes = oracle.four_cliques_filter_counts(g, sk)
        bha, bho, bsizes = _brute_filter_counts(g, sk)
        assert np.array_equal(ha, bha) and np.array_equal(ho, bho) and sizes == bsizes


def test_filter_counts_cover_every_triangle_once():
    # one (edge, w) per triangle: at its two lowest-ranked vertices
    for g in (pggen.rmat(10, 16, seed=2), pggen.er(500, 20, seed=1), pggen.complete(30),
              pggen.disjoint_union(pggen.complete(12), pggen.star(40), pggen.er(80, 9, seed=3))):
        sk = oracle.build_sketches(oracle.oriented(g), oracle.KIND_BF, 128, 1, seed=4)
        ha, ho, _ = oracle.four_cliques_filter_counts(g, sk)
        assert int(ha.sum()) == int(ho.sum()) == oracle.exact_tc_listing(g)
    sk = oracle.build_sketches(oracle.oriented(pggen.complete(30)), oracle.KIND_BF, 128, 1, seed=4)
    assert int(oracle.four_cliques_filter_counts(pggen.complete(30), sk)[0].sum()) == math.comb(30, 3)


@pytest.mark.parametrize("b", [1, 2])
def test_filter_limit_estimate_exact_when_hashes_are_injective(b):
    # disjoint bit sets per vertex: c = b |N+_w cap C3|, so the limit estimator c / b is exact
    g = pggen.er(200, 24, seed=2)
    B = 1 << 20
    seed = _injective_seed(g.n, B, b)
    sk = oracle.build_sketches(oracle.oriented(g), oracle.KIND_BF, B, b, seed)
    exact = oracle.four_cliques(g)
    assert exact > 0 and oracle.four_cliques_estimate(g, sk, "l") == float(exact)
    # and the logarithmic estimators sit close to it with so few ones per filter
    for est in ("and", "pap"):
        assert abs(oracle.four_cliques_estimate(g, sk, est) - exact) < 1e-3 * exact


def test_filter_estimates_on_complete_graph_closed_form():
    # K_n with an injective hash: the limit estimate is C(n, 4)
    for n in (6, 11, 17):
        g = pggen.complete(n)
        B = 1 << 16
        seed = _injective_seed(n, B, 1)
        sk = oracle.build_sketches(oracle.oriented(g), oracle.KIND_BF, B, 1, seed)
        assert oracle.four_cliques_estimate(g, sk, "l") == float(math.comb(n, 4))


def test_filter_or_estimate_uses_set_sizes():
    # OR: sum over (edge, w) of |N+_w| + |C3| + (B/b) ln(1 - c~_or/B); with an
    # injective hash, c_or = b |N+_w cup C3| and the estimate tends to the exact count
    g = pggen.er(200, 24, seed=2)
    B = 1 << 20
    seed = _injective_seed(g.n, B, 1)
    sk = oracle.build_sketches(oracle.oriented(g), oracle.KIND_BF, B, 1, seed)
    exact = oracle.four_cliques(g)
    assert abs(oracle.four_cliques_estimate(g, sk, "or") - exact) < 1e-2 * exact
