"""GPU parity of sketches of the degree-oriented sets N+_v (Listing "lst:tc")
and the oriented triangle-count estimate, through the C ABI, against the
oracle: rows and counts bit for bit, estimates within 1e-6 relative, the
triangle count within 1e-9 relative (FP64 summation order only)."""
import math
import sys

import numpy as np
import pytest

import oracle
import pggen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2208_11469_amd as pg  # noqa: E402

RTOL = 1e-6


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
    "er4096": lambda: pggen.er(4096, 16, seed=1),
    "rmat10": lambda: pggen.rmat(10, 16, seed=2),
    "rmat12": lambda: pggen.rmat(12, 16, seed=1),
    "hub": lambda: pggen.disjoint_union(pggen.star(6000), pggen.er(2000, 10, seed=3), pggen.complete(30)),
    "k2200": lambda: pggen.complete(2200),  # oriented degrees up to 2199: the heavy build tier
    "isolated": lambda: pggen.from_pairs(50, [], []),
    "single_edge": lambda: pggen.from_pairs(3, [0], [2]),
}
_CACHE = {}


def graph(name):
    if name not in _CACHE:
        _CACHE[name] = GRAPHS[name]()
    return _CACHE[name]


def np_(t):
    return t.detach().cpu().numpy()


def _close(got, want, rtol=RTOL, atol=1e-12):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    assert got.shape == want.shape
    err = np.abs(got - want)
    bad = err > atol + rtol * np.abs(want)
    assert not bad.any(), f"{bad.sum()} mismatches, worst {err.max()} at {np.argmax(err)}"


def _oracle_raw(ref, est, u, v):
    c = ref.counts(u, v)
    if ref.kind == oracle.KIND_BF:
        return c[1] if est == "or" else c[0]
    if ref.kind == oracle.KIND_KH:
        return c
    return c[2] if est == "1h_lit" else c[0]


KIND_OF = {"bf": oracle.KIND_BF, "kh": oracle.KIND_KH, "1h": oracle.KIND_1H}
CASES = [
    ("rmat12", "bf", 320, 1, ("and", "l", "or", "pap")),  # line-packed rows, slab triangle count
    ("er4096", "bf", 2048, 2, ("and", "or")),             # W = 32: the general paths
    ("hub", "bf", 256, 3, ("and",)),
    ("k2200", "bf", 512, 1, ("and", "l")),
    ("rmat12", "kh", 32, 1, ("kh",)),
    ("hub", "1h", 32, 1, ("1h", "1h_lit")),
    ("rmat10", "1h", 64, 1, ("1h",)),
    ("isolated", "bf", 256, 1, ("and",)),
    ("single_edge", "kh", 8, 1, ("kh",)),
]


@pytest.mark.parametrize("name,kind,size,b,ests", CASES)
def test_oriented_sketches_match_oracle(ctx, name, kind, size, b, ests):
    g = graph(name)
    say(f"oriented {name} n={g.n} {kind} size={size} b={b}")
    dg = pg.Graph(ctx, g.offsets, g.adj, validate=True)
    sk = dg.build_sketches(kind, size, b, seed=13, oriented=True)
    assert sk.oriented and sk.kind == pg.KINDS[kind]
    o = oracle.oriented(g)
    ref = oracle.build_sketches(o, KIND_OF[kind], size, b, seed=13)
    rows, pc = sk.export()
    torch.cuda.synchronize()
    if kind == "bf":
        assert np.array_equal(np_(rows), ref.words.view(np.uint8).reshape(g.n, size // 8))
        assert np.array_equal(np_(pc).astype(np.uint32), ref.pc)
    else:
        assert np.array_equal(np_(rows), ref.sig.view(np.uint8).reshape(g.n, 4 * size))
    eu, ev = oracle.upper_edges(g)
    for est in ests:
        say(f"  estimator {est}")
        e_gpu, r_gpu = sk.intersect(est)
        torch.cuda.synchronize()
        assert np.array_equal(np_(r_gpu).astype(np.uint32), _oracle_raw(ref, est, eu, ev))
        _close(np_(e_gpu), ref.estimate(eu, ev, est))
        _close([sk.tc(est)], [oracle.tc_oriented(g, ref, est)], rtol=1e-9)
    # rebuilding in place gives the same rows
    sk.rebuild()
    rows2, _ = sk.export()
    torch.cuda.synchronize()
    assert torch.equal(rows, rows2)
    sk.close()
    dg.close()


def test_oriented_exact_when_lossless(ctx):
    """1-hash with k >= 2 max d+ estimates every |N+_u cap N+_v| exactly, so the
    oriented estimate equals the exact triangle count."""
    g = graph("rmat10")
    dg = pg.Graph(ctx, g.offsets, g.adj)
    k = 2 * int(oracle.oriented(g).degrees().max())
    sk = dg.build_sketches("1h", k, seed=3, oriented=True)
    assert sk.tc("1h") == float(dg.exact_tc())
    sk.close()
    dg.close()


def test_oriented_rejects_calls_defined_on_full_neighbourhoods(ctx):
    g = graph("rmat10")
    dg = pg.Graph(ctx, g.offsets, g.adj)
    sk = dg.build_sketches("bf", 256, 1, seed=1, oriented=True)
    for call in (lambda: sk.cc("and"), lambda: sk.jaccard("and"), lambda: sk.similarity("and", "overlap"),
                 lambda: sk.jarvis_patrick("and", "cn", 1.0), lambda: pg.Server(dg, [sk])):
        with pytest.raises(pg.PGError) as err:
            call()
        assert err.value.code == pg.PG_E_UNSUPPORTED
    # the plain sketch set of the same graph still works beside it
    plain = dg.build_sketches("bf", 256, 1, seed=1)
    ref = oracle.build_sketches(g, oracle.KIND_BF, 256, 1, seed=1)
    _close([plain.tc("and")], [oracle.tc(ref, "and")], rtol=1e-9)
    plain.close()
    sk.close()
    dg.close()


@pytest.fixture(scope="module")
def g20():
    say("generating R-MAT scale 20, edge factor 16")
    return pggen.rmat(20, 16, seed=1)


@pytest.mark.timeout(600)
def test_full_size_rmat20_oriented(ctx, g20):
    g = g20
    dg = pg.Graph(ctx, g.offsets, g.adj)
    B = dg.bits_for_budget(0.33)
    o = oracle.oriented(g)
    assert int(o.degrees().max()) <= math.isqrt(g.nnz)
    say(f"full size oriented BF-{B}")
    sk = dg.build_sketches("bf", B, 1, seed=1, oriented=True)
    ref = oracle.build_sketches(o, oracle.KIND_BF, B, 1, seed=1)
    rows, pc = sk.export()
    torch.cuda.synchronize()
    assert np.array_equal(np_(rows), ref.words.view(np.uint8).reshape(g.n, B // 8))
    assert np.array_equal(np_(pc).astype(np.uint32), ref.pc)
    _close([sk.tc("and")], [oracle.tc_oriented(g, ref, "and")], rtol=1e-9)
    sk.close()
    say("full size oriented k-hash k=32")
    sk = dg.build_sketches("kh", 32, seed=1, oriented=True)
    ref = oracle.build_sketches(o, oracle.KIND_KH, 32, seed=1)
    rows, _ = sk.export()
    torch.cuda.synchronize()
    assert np.array_equal(np_(rows), ref.sig.view(np.uint8).reshape(g.n, 128))
    _close([sk.tc("kh")], [oracle.tc_oriented(g, ref, "kh")], rtol=1e-9)
    sk.close()
    dg.close()
