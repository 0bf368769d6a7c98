"""GPU parity of the KMV estimators on 1-hash rows (Section "Beyond Bloom
Filter and MinHash"), through the C ABI, against the oracle: union sizes
min(k, |M_u u M_v|) bit for bit; estimates within 1e-6 relative (the same FP64
operations in the same order on both sides); triangle counts within 1e-9 and
clustering coefficients within 1e-6 plus one FP32 rounding."""
import sys

import numpy as np
import pytest

import oracle
import pggen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2208_11469_amd as pg  # noqa: E402

RTOL = 1e-6
ESTS = ("kmv", "kmv_est")


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pg.Context(0)
    yield c
    c.close()


def np_(t):
    return t.detach().cpu().numpy()


def _close(got, want, rtol=RTOL, atol=1e-9):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    assert got.shape == want.shape
    err = np.abs(got - want)
    bad = err > atol + rtol * np.abs(want)
    assert not bad.any(), f"{bad.sum()} mismatches, worst {err.max()} at {np.argmax(err)}"


GRAPHS = {
    "er4096": lambda: pggen.er(4096, 16, seed=1),
    "rmat12": lambda: pggen.rmat(12, 16, seed=1),
    "hub": lambda: pggen.disjoint_union(pggen.star(3000), pggen.er(1500, 10, seed=3), pggen.complete(30)),
    "er_small": lambda: pggen.er(600, 5, seed=9),
    "isolated": lambda: pggen.from_pairs(50, [], []),
    "single_edge": lambda: pggen.from_pairs(3, [0], [2]),
}
CASES = [("er4096", 32), ("er4096", 64), ("rmat12", 32), ("hub", 16), ("er_small", 2), ("isolated", 8),
         ("single_edge", 4)]


@pytest.mark.parametrize("name,k", CASES)
def test_kmv_matches_oracle(ctx, name, k):
    g = GRAPHS[name]()
    say(f"kmv {name} n={g.n} k={k}")
    dg = pg.Graph(ctx, g.offsets, g.adj, validate=True)
    sk = dg.build_sketches("1h", k, seed=21)
    ref = oracle.build_sketches(g, oracle.KIND_1H, k, 1, seed=21)
    eu, ev = oracle.upper_edges(g)
    rng = np.random.default_rng(k)
    ru = rng.integers(0, g.n, 2000).astype(np.int32)
    rv = rng.integers(0, g.n, 2000).astype(np.int32)
    ru[:5] = rv[:5]
    dev = torch.device("cuda", 0)
    tu, tv = torch.from_numpy(ru).to(dev), torch.from_numpy(rv).to(dev)
    for est in ESTS:
        say(f"  {est}")
        e_gpu, r_gpu = sk.intersect(est)
        torch.cuda.synchronize()
        assert np.array_equal(np_(r_gpu).astype(np.uint32), ref.counts(eu, ev)[1])
        _close(np_(e_gpu), ref.estimate(eu, ev, est))
        e2, r2 = sk.intersect(est, tu, tv)
        torch.cuda.synchronize()
        assert np.array_equal(np_(r2).astype(np.uint32), ref.counts(ru, rv)[1])
        _close(np_(e2), ref.estimate(ru, rv, est))
        _close([sk.tc(est)], [oracle.tc(ref, est)], rtol=1e-9)
        cc = sk.cc(est)
        torch.cuda.synchronize()
        _close(np_(cc), oracle.cc(ref, est), rtol=RTOL + 2.0**-23, atol=1e-30)
    sk.close()
    dg.close()


def test_kmv_lossless_rows_give_exact_counts(ctx):
    g = GRAPHS["er_small"]()
    dg = pg.Graph(ctx, g.offsets, g.adj)
    k = int(g.degrees().max()) + 1
    sk = dg.build_sketches("1h", k, seed=4)
    for est in ESTS:
        e, _ = sk.intersect(est)
        torch.cuda.synchronize()
        assert np.array_equal(np_(e), np_(dg.exact_intersect()).astype(np.float64))
        assert sk.tc(est) == float(dg.exact_tc())
    sk.close()
    dg.close()


def test_kmv_oriented_tc(ctx):
    g = GRAPHS["rmat12"]()
    dg = pg.Graph(ctx, g.offsets, g.adj)
    sk = dg.build_sketches("1h", 32, seed=5, oriented=True)
    ref = oracle.build_sketches(oracle.oriented(g), oracle.KIND_1H, 32, 1, seed=5)
    for est in ESTS:
        _close([sk.tc(est)], [oracle.tc_oriented(g, ref, est)], rtol=1e-9)
    sk.close()
    dg.close()


@pytest.mark.timeout(600)
def test_full_size_rmat20_kmv_samples(ctx):
    """Full size: sampled edge estimates against the oracle's rows of their
    endpoints, and the triangle count as one third of the per-edge sum."""
    say("generating R-MAT scale 20, edge factor 16")
    g = pggen.rmat(20, 16, seed=1)
    dg = pg.Graph(ctx, g.offsets, g.adj)
    sk = dg.build_sketches("1h", 32, seed=1)
    eu_t, ev_t = dg.upper_edges()
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([rng.integers(0, dg.m, 3000), np.arange(100)]))
    idx_t = torch.from_numpy(idx).to(eu_t.device)
    su = eu_t[idx_t].cpu().numpy().astype(np.int64)
    sv = ev_t[idx_t].cpu().numpy().astype(np.int64)
    ends = np.unique(np.concatenate([su, sv]))
    ref = oracle.sketch_rows(g, ends, oracle.KIND_1H, 32, 1, 1)
    iu, iv = np.searchsorted(ends, su), np.searchsorted(ends, sv)
    for est in ESTS:
        say(f"full size {est}")
        e, _ = sk.intersect(est)
        torch.cuda.synchronize()
        _close(np_(e)[idx], ref.estimate(iu, iv, est))
        _close([sk.tc(est)], [float(e.sum().item()) / 3.0], rtol=1e-9)
    sk.close()
    dg.close()
