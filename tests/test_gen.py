"""Input generator: published SplitMix64 vectors and CSR invariants."""
import math

import numpy as np
import pytest

import pggen
from conftest import golden


def test_splitmix64_published_vector():
    want = [int(x) for x in golden("splitmix64_seed1234567.txt")]
    assert [pggen.splitmix64(1234567, i) for i in range(5)] == want


def _check_csr(g):
    off, adj = g.offsets, g.adj
    assert off.dtype == np.int32 and adj.dtype == np.int32
    assert off[0] == 0 and off[-1] == adj.shape[0]
    assert np.all(np.diff(off) >= 0)
    src = np.repeat(np.arange(g.n), np.diff(off))
    assert np.all(adj >= 0) and np.all(adj < g.n)
    assert not np.any(src == adj), "self-loop"
    # strictly ascending inside each neighbourhood
    same = src[1:] == src[:-1]
    assert np.all(adj[1:][same] > adj[:-1][same])
    # symmetric: the arc multiset equals its transpose
    fwd = src.astype(np.int64) * g.n + adj
    rev = adj.astype(np.int64) * g.n + src
    assert np.array_equal(np.sort(fwd), np.sort(rev))


@pytest.mark.parametrize("make", [
    lambda: pggen.er(4096, 16, seed=1),
    lambda: pggen.er(300, 40, seed=7),
    lambda: pggen.rmat(12, 16, seed=1),
    lambda: pggen.rmat(0, 16, seed=3, n=1000),
    lambda: pggen.complete(7), lambda: pggen.star(9), lambda: pggen.cycle(5), lambda: pggen.wheel(6),
    lambda: pggen.complete_bipartite(3, 4), lambda: pggen.friendship(4),
    lambda: pggen.disjoint_union(pggen.complete(4), pggen.cycle(6), pggen.from_pairs(3, [], [])),
])
def test_csr_invariants(make):
    _check_csr(make())


def test_er_edge_count_matches_gnp():
    # E[m] = C(n,2) p with p = 16/(n-1), i.e. 8n; sd = sqrt(C(n,2) p (1-p))
    n = 4096
    p = 16 / (n - 1)
    mean = n * (n - 1) / 2 * p
    sd = math.sqrt(n * (n - 1) / 2 * p * (1 - p))
    ms = [pggen.er(n, 16, seed=s).m for s in range(1, 6)]
    assert abs(np.mean(ms) - mean) < 4 * sd / math.sqrt(len(ms))


def test_er_degree_distribution_is_binomial():
    n = 2000
    g = pggen.er(n, 10, seed=3)
    d = g.degrees()
    assert abs(d.mean() - 10) < 0.5
    assert abs(d.var() - 10 * (1 - 10 / (n - 1))) < 1.5


def test_rmat_quadrant_skew():
    # with a = 0.57 the low IDs collect most edges: vertex 0 is the hub and the
    # lower half of the ID space holds about a + b = 0.76 of the endpoints
    g = pggen.rmat(12, 16, seed=2)
    d = g.degrees()
    assert d.argmax() == 0
    frac_low = d[: g.n // 2].sum() / d.sum()
    assert 0.70 < frac_low < 0.82


def test_rmat_rejection_keeps_ids_in_range_and_is_seeded():
    g1 = pggen.rmat(0, 16, seed=5, n=777)
    g2 = pggen.rmat(0, 16, seed=5, n=777)
    g3 = pggen.rmat(0, 16, seed=6, n=777)
    assert g1.n == 777 and g1.adj.max() < 777
    assert np.array_equal(g1.adj, g2.adj) and not np.array_equal(g1.adj, g3.adj)


def test_query_trace_pairs_distinct_and_sized():
    tr = pggen.query_trace(1000, 50, rate_hz=100.0, seed=3)
    for r in tr:
        assert 1 <= r.u.shape[0] <= 65536
        assert np.all(r.u != r.v) and r.u.max() < 1000 and r.v.max() < 1000
    arr = [r.arrival_s for r in tr]
    assert all(b >= a for a, b in zip(arr, arr[1:]))
