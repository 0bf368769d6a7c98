"""Pins for the oracle's KMV estimators (Section "Beyond Bloom Filter and
MinHash", Appendix "KMV Sketches"): keys against the C oracle's MinHash key,
exactness where the rows hold whole sets, the union-sketch construction against
the KMV of the union itself, the Beta law of the k-th smallest hash
(Eq. "est_ss_kmv" and its Proposition), unbiasedness of the union estimate,
and the deviation probability of the intersection estimate with exact sizes."""
import numpy as np
import pytest
from scipy import stats

import oracle
import pggen


def test_vector_keys_match_the_scalar_key():
    a, c = oracle.hash_consts(oracle.KIND_1H, 17, 1)
    xs = np.concatenate([np.arange(0, 3000), [2**31 - 1, 123456789]])
    want = np.array([oracle.mh_key(int(a[0]), int(c[0]), int(x)) for x in xs], dtype=np.uint64)
    assert np.array_equal(oracle.mh_keys(int(a[0]), int(c[0]), xs), want)


def test_hash_range_and_order():
    keys = np.array([0, 1, 2047, 2048, 2**63, 2**64 - 1], dtype=np.uint64)
    h = oracle.kmv_hash(keys)
    assert h[0] == 2.0**-53 and h[-1] == 1.0
    assert np.all(np.diff(h) >= 0) and np.all((h > 0) & (h <= 1))


def test_exact_when_rows_hold_whole_sets():
    g = pggen.er(400, 6, seed=8)
    k = int(g.degrees().max()) + 1  # every row holds its whole set
    sk = oracle.build_sketches(g, oracle.KIND_1H, k, 1, seed=2)
    eu, ev = oracle.upper_edges(g)
    exact = oracle.exact_pairs(g, eu, ev).astype(np.float64)
    for est in ("kmv", "kmv_est"):
        assert np.array_equal(sk.estimate(eu, ev, est), exact), est


def test_empty_sets_give_zero():
    g = pggen.disjoint_union(pggen.star(100), pggen.from_pairs(3, [], []))
    sk = oracle.build_sketches(g, oracle.KIND_1H, 8, 1, seed=1)
    for est in ("kmv", "kmv_est"):
        assert list(sk.estimate([0, 101, 101], [101, 0, 102], est)) == [0.0, 0.0, 0.0]


def test_union_sketch_is_the_kmv_of_the_union():
    rng = np.random.default_rng(4)
    for trial in range(200):
        x = rng.choice(5000, size=rng.integers(1, 300), replace=False)
        y = rng.choice(5000, size=rng.integers(1, 300), replace=False)
        k = int(rng.integers(2, 64))
        seed = 1000 + trial
        ku = np.union1d(oracle.kmv_of_set(x, k, seed), oracle.kmv_of_set(y, k, seed))[:k]
        assert np.array_equal(ku, oracle.kmv_of_set(np.union1d(x, y), k, seed))


def _union_hashes(k, trials, x, y):
    out = np.empty(trials)
    for t in range(trials):
        ku = np.union1d(oracle.kmv_of_set(x, k, t + 1), oracle.kmv_of_set(y, k, t + 1))
        out[t] = ku[k - 1]
    return out


def test_kth_smallest_hash_is_beta_distributed():
    # |X u Y| = 400, k = 24: the k-th smallest of N uniforms is Beta(k, N - k + 1)
    x, y = np.arange(0, 250), np.arange(150, 400)
    k, N = 24, 400
    h = _union_hashes(k, 3000, x, y)
    assert stats.kstest(h, stats.beta(k, N - k + 1).cdf).pvalue > 1e-3


def test_union_estimate_is_unbiased():
    x, y = np.arange(0, 700), np.arange(500, 1000)
    k, N, trials = 40, 1000, 3000
    est = (k - 1) / _union_hashes(k, trials, x, y)
    # (k-1)/U_(k) is unbiased for N with variance N (N - k + 1) / (k - 2)
    sd = np.sqrt(N * (N - k + 1) / (k - 2) / trials)
    assert abs(est.mean() - N) < 4 * sd


def test_intersection_deviation_probability():
    """With exact sizes, |I^ - I| = |U^ - |X u Y||, so
    P(|I^ - I| <= t) = I_u(k, N-k+1) - I_l(k, N-k+1), u = (k-1)/(N-t),
    l = (k-1)/(N+t) (the Proposition of Appendix "KMV Sketches", read with <=)."""
    x, y = np.arange(0, 300), np.arange(200, 520)
    k, N, I = 32, 520, 100
    trials = 3000
    def row_keys(xs, seed):
        a, c = oracle.hash_consts(oracle.KIND_1H, seed, 1)
        return np.sort(oracle.mh_keys(int(a[0]), int(c[0]), xs))[:k]

    got = np.array([oracle.kmv_intersection(row_keys(x, t + 1), row_keys(y, t + 1), k, x.shape[0], y.shape[0], True)
                    for t in range(trials)])
    beta = stats.beta(k, N - k + 1)
    for t in (20.0, 60.0, 120.0):
        p = beta.cdf((k - 1) / (N - t)) - beta.cdf((k - 1) / (N + t))
        emp = np.mean(np.abs(got - I) <= t)
        assert abs(emp - p) < 4 * np.sqrt(p * (1 - p) / trials) + 1e-3, (t, emp, p)
