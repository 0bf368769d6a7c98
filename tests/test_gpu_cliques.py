"""GPU parity of 4-clique counting (Listing "lst:fcl"), exact and from Bloom
filters of the oriented sets, through the C ABI, against the oracle: the exact
and membership counts are integers and must match bit for bit; the estimates
from sketch intersections (filter of N+_w against a filter of C3) are FP64
sums that must match within 1e-9 relative (reassociation only), and bit for
bit for the limit estimator with b <= 2 (sums of multiples of 1/2)."""
import math
import sys

import numpy as np
import pytest

import oracle
import pggen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2208_11469_amd as pg  # noqa: E402


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


GRAPHS = {
    "k5": lambda: pggen.complete(5),
    "k60": lambda: pggen.complete(60),
    "er4096": lambda: pggen.er(4096, 16, seed=1),
    "rmat12": lambda: pggen.rmat(12, 16, seed=1),
    "rmat14": lambda: pggen.rmat(14, 16, seed=2),
    "hub": lambda: pggen.disjoint_union(pggen.star(6000), pggen.er(2000, 10, seed=3), pggen.complete(30)),
    "no_k4": lambda: pggen.disjoint_union(pggen.wheel(8), pggen.friendship(6), pggen.complete_bipartite(9, 11)),
    "isolated": lambda: pggen.from_pairs(50, [], []),
}
# (graph, B, b) for the filter estimate
BF = {"k5": (64, 1), "k60": (128, 2), "er4096": (256, 1), "rmat12": (320, 2), "rmat14": (2048, 1),
      "hub": (192, 3), "no_k4": (64, 1), "isolated": (64, 1)}


@pytest.mark.parametrize("name", list(GRAPHS))
def test_four_cliques_match_oracle(ctx, name):
    g = GRAPHS[name]()
    say(f"4-cliques {name} n={g.n} nnz={g.nnz}")
    dg = pg.Graph(ctx, g.offsets, g.adj, validate=True)
    exact = dg.exact_four_cliques()
    want = oracle.four_cliques(g)
    assert exact == want
    if name == "k5":
        assert exact == 5
    if name == "k60":
        assert exact == math.comb(60, 4)
    if name in ("no_k4", "isolated"):
        assert exact == 0
    B, b = BF[name]
    sk = dg.build_sketches("bf", B, b, seed=7, oriented=True)
    ref = oracle.build_sketches(oracle.oriented(g), oracle.KIND_BF, B, b, seed=7)
    est = sk.four_cliques()
    assert est == oracle.four_cliques_bf(g, ref)
    assert est >= exact
    sk.close()
    dg.close()


def test_four_cliques_reject_wrong_sketches(ctx):
    g = GRAPHS["rmat12"]()
    dg = pg.Graph(ctx, g.offsets, g.adj)
    for kind, oriented in (("bf", False), ("kh", True), ("1h", True)):
        sk = dg.build_sketches(kind, 64, 1, seed=1, oriented=oriented)
        with pytest.raises(pg.PGError) as err:
            sk.four_cliques()
        assert err.value.code == pg.PG_E_INVALID
        sk.close()
    dg.close()


def test_four_cliques_refuse_oversized_triangle_lists(ctx):
    # K_4200: oriented degrees up to 4199 exceed the on-chip C3 buffer
    g = pggen.complete(4200)
    dg = pg.Graph(ctx, g.offsets, g.adj)
    with pytest.raises(pg.PGError) as err:
        dg.exact_four_cliques()
    assert err.value.code == pg.PG_E_UNSUPPORTED
    dg.close()


@pytest.mark.timeout(600)
def test_rmat18_four_cliques(ctx):
    say("generating R-MAT scale 18, edge factor 16")
    g = pggen.rmat(18, 16, seed=1)
    dg = pg.Graph(ctx, g.offsets, g.adj)
    B = dg.bits_for_budget(0.33)
    say(f"exact 4-cliques, m={dg.m}")
    assert dg.exact_four_cliques() == oracle.four_cliques(g)
    say(f"BF-{B} 4-cliques")
    sk = dg.build_sketches("bf", B, 1, seed=1, oriented=True)
    ref = oracle.build_sketches(oracle.oriented(g), oracle.KIND_BF, B, 1, seed=1)
    assert sk.four_cliques() == oracle.four_cliques_bf(g, ref)
    sk.close()
    dg.close()


FILTER_ESTS = ("and", "l", "pap", "or")


def _check_estimates(g, sk, ref, b):
    for est in FILTER_ESTS:
        got = sk.four_cliques_estimate(est)
        want = oracle.four_cliques_estimate(g, ref, est)
        if est == "l" and b <= 2:
            assert got == want, (est, got, want)
        else:
            assert abs(got - want) <= 1e-9 * max(abs(want), 1.0), (est, got, want)
        assert sk.four_cliques_estimate(est) == got  # independent of scheduling


FILTER_GRAPHS = dict(GRAPHS, k1200=lambda: pggen.complete(1200))  # C3 of up to 1198 elements
FILTER_BF = dict(BF, k1200=(320, 1))


@pytest.mark.parametrize("name", list(FILTER_GRAPHS))
def test_four_clique_filter_estimates_match_oracle(ctx, name):
    g = FILTER_GRAPHS[name]()
    B, b = FILTER_BF[name]
    say(f"4-clique filter estimates {name} B={B} b={b}")
    dg = pg.Graph(ctx, g.offsets, g.adj)
    sk = dg.build_sketches("bf", B, b, seed=7, oriented=True)
    ref = oracle.build_sketches(oracle.oriented(g), oracle.KIND_BF, B, b, seed=7)
    _check_estimates(g, sk, ref, b)
    if name in ("no_k4", "isolated"):
        assert sk.four_cliques_estimate("l") == oracle.four_cliques_estimate(g, ref, "l")
    sk.close()
    dg.close()


def test_four_clique_filter_limit_exact_with_injective_hash(ctx):
    # every vertex on its own bit: c = |N+_w cap C3| and the limit estimate is the exact count
    g = pggen.er(100, 20, seed=4)
    B = 4096
    for seed in range(1, 400):
        a, c = oracle.hash_consts(oracle.KIND_BF, seed, 1)
        if len({oracle.bf_index(int(a[0]), int(c[0]), x, B) for x in range(g.n)}) == g.n:
            break
    else:
        raise AssertionError("no injective seed found")
    dg = pg.Graph(ctx, g.offsets, g.adj)
    sk = dg.build_sketches("bf", B, 1, seed=seed, oriented=True)
    exact = dg.exact_four_cliques()
    assert exact > 0 and sk.four_cliques_estimate("l") == float(exact)
    sk.close()
    dg.close()


def test_four_clique_filter_estimates_refusals(ctx):
    g = GRAPHS["rmat12"]()
    dg = pg.Graph(ctx, g.offsets, g.adj)
    for kind, oriented in (("bf", False), ("kh", True)):
        sk = dg.build_sketches(kind, 64, 1, seed=1, oriented=oriented)
        with pytest.raises(pg.PGError) as err:
            sk.four_cliques_estimate("and")
        assert err.value.code == pg.PG_E_INVALID
        sk.close()
    sk = dg.build_sketches("bf", 256, 1, seed=1, oriented=True)
    with pytest.raises(pg.PGError) as err:
        sk.four_cliques_estimate("kh")
    assert err.value.code == pg.PG_E_INVALID
    sk.close()
    dg.close()
    # K_6100 with 4096-bit filters: the table (32.8 KB) and four C3 buffers of
    # oriented degree up to 6099 (24.9 KB each) exceed 128 KiB of LDS
    g = pggen.complete(6100)
    dg = pg.Graph(ctx, g.offsets, g.adj)
    sk = dg.build_sketches("bf", 4096, 1, seed=1, oriented=True)
    with pytest.raises(pg.PGError) as err:
        sk.four_cliques_estimate("and")
    assert err.value.code == pg.PG_E_UNSUPPORTED
    sk.close()
    dg.close()


@pytest.mark.timeout(600)
def test_rmat18_four_clique_filter_estimates(ctx):
    say("generating R-MAT scale 18, edge factor 16")
    g = pggen.rmat(18, 16, seed=1)
    dg = pg.Graph(ctx, g.offsets, g.adj)
    B = dg.bits_for_budget(0.33)
    say(f"BF-{B} 4-clique filter estimates")
    sk = dg.build_sketches("bf", B, 1, seed=1, oriented=True)
    ref = oracle.build_sketches(oracle.oriented(g), oracle.KIND_BF, B, 1, seed=1)
    _check_estimates(g, sk, ref, 1)
    sk.close()
    dg.close()
