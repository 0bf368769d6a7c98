"""Pins for the oracle's sketches and estimators.

What fixes them, beyond the oracle's own code:
  * the published SplitMix64 vector (the generator behind every hash constant);
  * invariants any correct Bloom filter / MinHash must satisfy;
  * closed values of the estimator formulas;
  * convergence to the exact count when hashes become injective (Appendix C,
    consistency as the filter grows; Section 4.4, 1-hash exact once k covers
    both sets);
  * the distributions the paper states: ones of a filter (Section 2.5),
    Bin(k, J) for k-hash (Section 4.3), Hypergeometric(|X u Y|, |X n Y|, k)
    for 1-hash (Section 4.4), the expectation sums of Appendix D and the MSE
    bound of Proposition "bound_int_BF".
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import pggen
from conftest import golden

KBF, KKH, K1H = oracle.KIND_BF, oracle.KIND_KH, oracle.KIND_1H


def test_oracle_splitmix64_published_vector():
    want = [int(x) for x in golden("splitmix64_seed1234567.txt")]
    assert [oracle.splitmix64(1234567, i) for i in range(5)] == want


def test_hash_constants_odd_and_seeded():
    for kind in (KBF, KKH, K1H):
        a, c = oracle.hash_consts(kind, 1, 64)
        assert np.all(a & np.uint64(1) == 1)
        assert len(set(a.tolist())) == 64 and len(set(c.tolist())) == 64
    a1, _ = oracle.hash_consts(KBF, 1, 4)
    a2, _ = oracle.hash_consts(KBF, 2, 4)
    a3, _ = oracle.hash_consts(KKH, 1, 4)
    assert not np.array_equal(a1, a2) and not np.array_equal(a1, a3)


@pytest.mark.parametrize("B", [64, 256, 320, 1024])
def test_bf_index_in_range_and_uniform(B):
    a, c = oracle.hash_consts(KBF, 11, 2)
    rng = np.random.default_rng(B)
    xs = rng.integers(0, 2**31, size=20000)
    idx = np.array([oracle.bf_index(int(a[0]), int(c[0]), int(x), B) for x in xs])
    assert idx.min() >= 0 and idx.max() < B
    counts = np.bincount(idx, minlength=B)
    chi2 = ((counts - len(xs) / B) ** 2 / (len(xs) / B)).sum()
    assert stats.chi2.sf(chi2, B - 1) > 1e-4


def test_mh_key_is_injective_on_ids():
    a, c = oracle.hash_consts(KKH, 5, 1)
    keys = {oracle.mh_key(int(a[0]), int(c[0]), x) for x in range(5000)}
    assert len(keys) == 5000


# ----------------------------------------------------------------- Bloom filters

@pytest.mark.parametrize("B,b", [(256, 1), (320, 2), (128, 3)])
def test_bf_invariants(B, b):
    g = pggen.rmat(10, 16, seed=4)
    sk = oracle.build_sketches(g, KBF, B, b, seed=9)
    d = g.degrees()
    ones = np.array([sum(bin(int(w)).count("1") for w in row) for row in sk.words])
    assert np.array_equal(ones, sk.pc)
    assert np.all(sk.pc <= np.minimum(b * d, B))
    assert np.all((sk.pc == 0) == (d == 0))
    eu, ev = oracle.upper_edges(g)
    ca, co = sk.counts(eu, ev)
    assert np.all(ca <= np.minimum(sk.pc[eu], sk.pc[ev]))
    assert np.array_equal(co.astype(np.int64), sk.pc[eu].astype(np.int64) + sk.pc[ev] - ca)
    # the AND of two filters contains the filter of the intersection (Section 4.2)
    for e in range(0, eu.shape[0], max(1, eu.shape[0] // 300)):
        inter = np.intersect1d(g.neighbours(eu[e]), g.neighbours(ev[e]))
        fi = oracle.bf_of_set(inter, B, b, 9)
        and_words = sk.words[eu[e]] & sk.words[ev[e]]
        assert np.all(fi & ~and_words == 0)
        assert ca[e] >= sum(bin(int(w)).count("1") for w in fi)
    # a vertex's filter is the filter of its neighbourhood
    for v in (0, 1, 17, g.n - 1):
        assert np.array_equal(sk.words[v], oracle.bf_of_set(g.neighbours(v), B, b, 9))


@pytest.mark.parametrize("B,b,size", [(256, 1, 20), (256, 2, 40), (320, 1, 100)])
def test_bf_expected_ones(B, b, size):
    # E[B_{X,1}] = B (1 - (1 - 1/B)^{b |X|}) (Section 2.5 / Appendix C)
    rng = np.random.default_rng(size)
    pcs = []
    for seed in range(1500):
        xs = rng.choice(2**31, size=size, replace=False)
        w = oracle.bf_of_set(xs, B, b, seed)
        pcs.append(sum(bin(int(x)).count("1") for x in w))
    pcs = np.array(pcs, dtype=np.float64)
    want = B * (1 - (1 - 1 / B) ** (b * size))
    se = pcs.std(ddof=1) / math.sqrt(len(pcs))
    assert abs(pcs.mean() - want) < 5 * se + 1e-9


def test_bf_estimator_closed_values():
    for B in (64, 256, 1024):
        for b in (1, 2, 4):
            assert oracle.est_bf_and([0], B, b)[0] == 0.0
            # c = B is moved to B - 1 (Appendix C): (B/b) ln B
            assert oracle.est_bf_and([B], B, b)[0] == pytest.approx(B / b * math.log(B), rel=1e-14)
            assert oracle.est_bf_limit([7], B, b)[0] == 7 / b
            assert oracle.est_bf_papapetrou([0], B, b)[0] == 0.0
        assert oracle.est_bf_and([1], B, 1)[0] == pytest.approx(-B * math.log(1 - 1 / B), rel=1e-14)
        # the existing estimator counts one element exactly for b = 1
        assert oracle.est_bf_papapetrou([1], B, 1)[0] == pytest.approx(1.0, rel=1e-14)
        # OR with an empty union: |X| + |Y|
        assert oracle.est_bf_or([0], [3], [4], B, 1)[0] == 7.0
    # the AND estimator exceeds the limit estimator (the log's series has only positive terms)
    c = np.arange(1, 200)
    assert np.all(oracle.est_bf_and(c, 256, 1) > oracle.est_bf_limit(c, 256, 1))


@pytest.mark.parametrize("size,B,b", [(40, 1024, 2), (30, 512, 1)])
def test_bf_single_set_estimator_unbiased_and_mse_bound(size, B, b):
    # Eq. "est_ss_bf" on one filter; Proposition "bound_int_BF" (which the paper
    # states also holds for this estimator) bounds its MSE.
    rng = np.random.default_rng(B + size)
    ests = []
    for seed in range(2000):
        xs = rng.choice(2**31, size=size, replace=False)
        w = oracle.bf_of_set(xs, B, b, 1000 + seed)
        ones = sum(bin(int(x)).count("1") for x in w)
        ests.append(oracle.est_bf_and([ones], B, b)[0])
    ests = np.array(ests)
    se = ests.std(ddof=1) / math.sqrt(len(ests))
    assert abs(ests.mean() - size) < 0.02 * size + 5 * se
    mse = np.mean((ests - size) ** 2)
    bound = math.exp(size * b / (B - 1)) * B / b**2 - B / b**2 - size / b
    assert mse <= 1.25 * bound


def _injective_seed(n, B, b):
    for seed in range(1, 200):
        a, c = oracle.hash_consts(KBF, seed, b)
        idx = {oracle.bf_index(int(a[i]), int(c[i]), x, B) for x in range(n) for i in range(b)}
        if len(idx) == n * b:
            return seed
    raise AssertionError("no injective seed found")


@pytest.mark.parametrize("b", [1, 2])
def test_bf_estimators_exact_when_hashes_injective(b):
    # Once every (vertex, hash) pair owns a private bit, AND counts b|X n Y| ones
    # and OR counts b|X u Y| ones, so the limit estimator is exact and AND, OR and
    # the existing estimator are within O(b I^2 / B) of the exact count.
    g = pggen.er(120, 12, seed=3)
    B = 1 << 20
    seed = _injective_seed(g.n, B, b)
    sk = oracle.build_sketches(g, KBF, B, b, seed=seed)
    eu, ev = oracle.upper_edges(g)
    inter = oracle.exact_pairs(g, eu, ev).astype(np.float64)
    ca, co = sk.counts(eu, ev)
    assert np.array_equal(ca, b * inter)
    assert np.array_equal(sk.estimate(eu, ev, "l"), inter)
    for est in ("and", "or", "pap"):
        assert np.max(np.abs(sk.estimate(eu, ev, est) - inter)) < 1e-2, est
    assert oracle.tc(sk, "l") == pytest.approx(oracle.exact_tc(g), rel=1e-12)


def test_bf_and_error_shrinks_as_filter_grows():
    g = pggen.er(500, 16, seed=2)
    eu, ev = oracle.upper_edges(g)
    inter = oracle.exact_pairs(g, eu, ev).astype(np.float64)
    errs = []
    for B in (128, 512, 2048, 8192):
        e = [np.mean(np.abs(oracle.build_sketches(g, KBF, B, 1, seed=s).estimate(eu, ev, "and") - inter))
             for s in range(3)]
        errs.append(np.mean(e))
    assert all(x > y for x, y in zip(errs, errs[1:])), errs
    assert errs[-1] < 0.05


# ----------------------------------------------------------------- k-hash MinHash

def test_khash_deterministic_cases():
    k = 32
    g = pggen.complete_bipartite(2, 9)  # vertices 0 and 1 share N = {2..10}
    sk = oracle.build_sketches(g, KKH, k, seed=3)
    assert sk.counts([0], [1])[0] == k
    assert sk.estimate([0], [1], "kh")[0] == 9.0
    eu, ev = oracle.upper_edges(g)
    assert np.all(sk.counts(eu, ev) == 0) and oracle.tc(sk, "kh") == 0.0
    st = oracle.build_sketches(pggen.star(12), KKH, k, seed=3)
    assert oracle.tc(st, "kh") == 0.0
    # every slot holds an element of the neighbourhood; empty -> bottom
    g2 = pggen.disjoint_union(pggen.rmat(8, 8, seed=1), pggen.from_pairs(2, [], []))
    s2 = oracle.build_sketches(g2, KKH, k, seed=4)
    for v in range(g2.n):
        nb = set(g2.neighbours(v).tolist())
        if nb:
            assert set(s2.sig[v].tolist()) <= nb
        else:
            assert np.all(s2.sig[v] == oracle.BOTTOM)


def test_khash_signature_is_argmin_and_spread():
    g = pggen.er(200, 30, seed=5)
    k = 16
    sk = oracle.build_sketches(g, KKH, k, seed=8)
    a, c = oracle.hash_consts(KKH, 8, k)
    for v in (0, 7, 199):
        nb = g.neighbours(v)
        for i in range(k):
            keys = [oracle.mh_key(int(a[i]), int(c[i]), int(x)) for x in nb]
            assert sk.sig[v, i] == nb[int(np.argmin(keys))]
    # with d = 30 and k = 16, the positions pick many different elements
    assert np.mean([len(set(r.tolist())) for r in sk.sig]) > 8


def _pair_sets(rng, nx, ny, ni):
    pool = rng.choice(2**31 - 1, size=nx + ny - ni, replace=False)
    X = pool[:nx]
    Y = np.concatenate([pool[:ni], pool[nx:]])
    return X, Y


def _pair_graph(X, Y):
    """Two vertices 0 and 1 whose neighbourhoods are X and Y (IDs shifted past 1)."""
    ids = np.unique(np.concatenate([X, Y]))
    remap = {int(x): i + 2 for i, x in enumerate(ids)}
    src = [0] * len(X) + [1] * len(Y)
    dst = [remap[int(x)] for x in X] + [remap[int(y)] for y in Y]
    return pggen.from_pairs(len(ids) + 2, src, dst)


def test_khash_binomial_mean_and_expectation_formula():
    # |M_X n M_Y| ~ Bin(k, J) (Section 4.3); E[I^_kH] is the binomial sum of Appendix D.
    k, nx, ny, ni = 32, 30, 30, 10
    J = ni / (nx + ny - ni)
    rng = np.random.default_rng(1)
    ss, ests = [], []
    for seed in range(300):
        X, Y = _pair_sets(rng, nx, ny, ni)
        g = _pair_graph(X, Y)
        sk = oracle.build_sketches(g, KKH, k, seed=seed)
        ss.append(sk.counts([0], [1])[0])
        ests.append(sk.estimate([0], [1], "kh")[0])
    ss, ests = np.array(ss, np.float64), np.array(ests)
    assert abs(ss.mean() / k - J) < 5 * math.sqrt(J * (1 - J) / (k * len(ss)))
    # dispersion of a binomial count
    assert 0.6 < ss.var(ddof=1) / (k * J * (1 - J)) < 1.5
    D = nx + ny
    expect = D * sum(math.comb(k, s) * J**s * (1 - J) ** (k - s) * s / (k + s) for s in range(k + 1))
    assert abs(ests.mean() - expect) < 5 * ests.std(ddof=1) / math.sqrt(len(ests))
    # Proposition "bound_int_mh": P(|I^ - I| >= t) <= 2 exp(-2 k t^2 / D^2)
    t = 9.0
    assert np.mean(np.abs(ests - ni) >= t) <= 2 * math.exp(-2 * k * t * t / D**2) + 0.02


# ----------------------------------------------------------------- 1-hash MinHash

def test_onehash_holds_bottom_k_in_hash_order():
    g = pggen.er(300, 40, seed=6)
    k = 16
    sk = oracle.build_sketches(g, K1H, k, seed=2)
    a, c = oracle.hash_consts(K1H, 2, 1)
    for v in (0, 5, 299):
        nb = g.neighbours(v)
        keys = np.array([oracle.mh_key(int(a[0]), int(c[0]), int(x)) for x in nb], dtype=np.uint64)
        order = np.argsort(keys, kind="stable")
        m = min(k, nb.shape[0])
        assert np.array_equal(sk.sig[v, :m], nb[order[:m]])
        assert np.all(sk.sig[v, m:] == oracle.BOTTOM)
        assert len(set(sk.sig[v, :m].tolist())) == m  # never duplicates


def test_onehash_exact_when_k_covers_degrees():
    # Section 4.4 / Appendix D: as k reaches |X u Y| the whole population is
    # sampled; k = 2 d_max covers every union (|X u Y| <= d_u + d_v).
    g = pggen.er(4096, 16, seed=1)
    k = 2 * int(g.degrees().max())
    sk = oracle.build_sketches(g, K1H, k, seed=1)
    eu, ev = oracle.upper_edges(g)
    inter = oracle.exact_pairs(g, eu, ev)
    assert np.allclose(sk.estimate(eu, ev, "1h"), inter, rtol=1e-12, atol=1e-12)
    assert oracle.tc(sk, "1h") == pytest.approx(oracle.exact_tc(g), rel=1e-12)
    assert np.allclose(oracle.cc(sk, "1h"), oracle.exact_cc(g), rtol=1e-12, atol=1e-12)
    # the literal reading divides by k instead and is not exact on small sets
    assert not np.allclose(sk.estimate(eu, ev, "1h_lit"), inter)


@pytest.mark.parametrize("n", [4, 10, 25])
def test_onehash_complete_graph_tc(n):
    sk = oracle.build_sketches(pggen.complete(n), K1H, 32, seed=n)
    assert oracle.tc(sk, "1h") == pytest.approx(math.comb(n, 3), rel=1e-12)


def test_onehash_hypergeometric_mean_and_expectation_formula():
    k, nx, ny, ni = 32, 100, 100, 40
    N = nx + ny - ni
    rng = np.random.default_rng(2)
    ss, kps, ests = [], [], []
    for seed in range(400):
        X, Y = _pair_sets(rng, nx, ny, ni)
        sk = oracle.build_sketches(_pair_graph(X, Y), K1H, k, seed=seed)
        su, kp, _ = sk.counts([0], [1])
        ss.append(su[0])
        kps.append(kp[0])
        ests.append(sk.estimate([0], [1], "1h")[0])
    assert set(kps) == {k}
    ss, ests = np.array(ss, np.float64), np.array(ests)
    mean = k * ni / N
    var = k * (ni / N) * (1 - ni / N) * (N - k) / (N - 1)
    assert abs(ss.mean() - mean) < 5 * math.sqrt(var / len(ss))
    assert 0.6 < ss.var(ddof=1) / var < 1.5
    D = nx + ny
    expect = D * sum(math.comb(ni, s) * math.comb(N - ni, k - s) / math.comb(N, k) * s / (k + s)
                     for s in range(k + 1))
    assert abs(ests.mean() - expect) < 5 * ests.std(ddof=1) / math.sqrt(len(ests))


# ----------------------------------------------------------------- outputs

def test_minhash_jaccard_equals_match_fraction_when_not_clamped():
    g = pggen.rmat(9, 8, seed=3)
    k = 32
    sk = oracle.build_sketches(g, KKH, k, seed=3)
    eu, ev = oracle.upper_edges(g)
    s = sk.counts(eu, ev).astype(np.float64)
    est = sk.estimate(eu, ev, "kh")
    jac = oracle.jaccard(sk, "kh", eu, ev)
    ok = est <= np.minimum(sk.deg[eu], sk.deg[ev])
    assert ok.mean() > 0.5
    assert np.allclose(jac[ok], s[ok] / k, rtol=1e-12, atol=1e-15)


def test_cc_and_tc_agree_with_per_edge_sum():
    g = pggen.rmat(10, 8, seed=5)
    sk = oracle.build_sketches(g, KBF, 256, 1, seed=5)
    eu, ev = oracle.upper_edges(g)
    est = sk.estimate(eu, ev, "and")
    d = g.degrees().astype(np.float64)
    cc = oracle.cc(sk, "and")
    # sum_v cc_v d_v (d_v - 1) adds the estimates of the arcs leaving vertices
    # with d_v >= 2; with every degree >= 2 that is each edge estimate twice
    au, av = oracle.arcs(g)
    keep = d[au] >= 2
    arc_sum = np.sum(sk.estimate(au[keep], av[keep], "and"))
    assert np.sum(cc * d * (d - 1)) == pytest.approx(arc_sum, rel=1e-12)
    g2 = pggen.complete(12)
    sk2 = oracle.build_sketches(g2, KBF, 256, 1, seed=5)
    e2u, e2v = oracle.upper_edges(g2)
    d2 = g2.degrees().astype(np.float64)
    assert np.sum(oracle.cc(sk2, "and") * d2 * (d2 - 1)) == pytest.approx(
        2 * sk2.estimate(e2u, e2v, "and").sum(), rel=1e-12)
    assert oracle.tc(sk, "and") == pytest.approx(est.sum() / 3, rel=1e-12)


def test_bits_for_budget_rule():
    g = pggen.rmat(12, 16, seed=1)
    for s in (0.1, 0.25, 0.33):
        B = oracle.bits_for_budget(g, s)
        assert B % 64 == 0 and B >= 64
        assert g.n * B <= s * 8 * g.csr_bytes() < g.n * (B + 64)
