"""GPU parity: the HIP library through its C ABI against the oracle.

Integers (sketch rows, popcounts, AND/OR/match counts, exact intersections and
triangle counts) must match bit for bit. FP64 estimates must be within 1e-6
relative of the FP64 oracle (observed: ~1e-15, rounding order only); FP32
outputs (CC, Jaccard) are checked at 1e-6 relative of the FP64 value, plus one
FP32 rounding.
"""
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


def _graphs():
    return {
        "er4096": lambda: pggen.er(4096, 16, seed=1),
        "rmat10": lambda: pggen.rmat(10, 16, seed=2),
        "rmat12": lambda: pggen.rmat(12, 16, seed=1),
        "rmat_n1000": lambda: pggen.rmat(0, 8, seed=4, n=1000),
        "hub": lambda: pggen.disjoint_union(pggen.star(6000), pggen.er(2000, 10, seed=3), pggen.complete(30)),
        "bigstar": lambda: pggen.star(200000),
        "k40": lambda: pggen.complete(40),
        "wheel7": lambda: pggen.wheel(7),
        "isolated": lambda: pggen.from_pairs(50, [], []),
        "single_edge": lambda: pggen.from_pairs(3, [0], [2]),
    }


_CACHE = {}


def graph(name):
    if name not in _CACHE:
        _CACHE[name] = _graphs()[name]()
    return _CACHE[name]


def dgraph(ctx, name, validate=True):
    g = graph(name)
    say(f"graph {name} n={g.n} nnz={g.nnz}")
    return g, pg.Graph(ctx, g.offsets, g.adj, validate=validate)


def np_(t):
    return t.detach().cpu().numpy()


def _rand_pairs(g, count, seed):
    rng = np.random.default_rng(seed)
    u = rng.integers(0, g.n, count).astype(np.int32)
    v = rng.integers(0, g.n, count).astype(np.int32)
    u[:5] = v[:5]  # a few u == v pairs
    return u, v


def _close(got, want, rtol=RTOL, atol=1e-12):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    assert got.shape == want.shape
    err = np.abs(got - want)
    bad = err > atol + rtol * np.abs(want)
    assert not bad.any(), f"{bad.sum()} mismatches, worst {err.max()} at {np.argmax(err)}"


def _close32(got, want):
    # FP32 rounded once from FP64: relative 2^-24 plus the 1e-6 tolerance
    _close(got, want, rtol=RTOL + 2.0**-23, atol=1e-30)


# ------------------------------------------------------------------ graph ingest

@pytest.mark.parametrize("name", list(_graphs()))
def test_graph_ingest(ctx, name):
    g, dg = dgraph(ctx, name)
    eu, ev = oracle.upper_edges(g)
    assert (dg.n, dg.nnz, dg.m) == (g.n, g.nnz, eu.shape[0])
    assert dg.max_degree == int(g.degrees().max(initial=0))
    du, dv = dg.upper_edges()
    assert np.array_equal(np_(du), eu) and np.array_equal(np_(dv), ev)
    dg.close()


def _expect_graph_error(ctx, n, off, adj, validate=True):
    with pytest.raises(pg.PGError) as ei:
        pg.Graph(ctx, np.asarray(off, np.int32), np.asarray(adj, np.int32), validate=validate)
    assert ei.value.code == pg.PG_E_GRAPH


def test_validation_rejects_malformed_csr(ctx):
    say("validation")
    # offsets not monotone / not ending at nnz / ID out of range: rejected even without PG_VALIDATE
    _expect_graph_error(ctx, 3, [0, 2, 1, 2], [1, 2], validate=False)
    _expect_graph_error(ctx, 3, [0, 1, 2, 3], [1, 0], validate=False)
    _expect_graph_error(ctx, 2, [0, 1, 2], [1, 7], validate=False)
    # structure checks under PG_VALIDATE
    _expect_graph_error(ctx, 2, [0, 1, 2], [0, 1])               # self-loops
    _expect_graph_error(ctx, 3, [0, 2, 3, 4], [2, 1, 0, 0])     # unsorted N_0
    _expect_graph_error(ctx, 2, [0, 2, 4], [1, 1, 0, 0])        # duplicates
    _expect_graph_error(ctx, 3, [0, 1, 2, 2], [1, 2])           # asymmetric
    # a good graph passes
    g = pggen.cycle(5)
    pg.Graph(ctx, g.offsets, g.adj, validate=True).close()


def test_empty_graph(ctx):
    say("empty graph n=0")
    dg = pg.Graph(ctx, np.zeros(1, np.int32), np.zeros(0, np.int32), validate=True)
    assert (dg.n, dg.m) == (0, 0)
    sk = dg.build_sketches("bf", 256, 1, seed=1)
    assert sk.tc("and") == 0.0
    assert dg.exact_tc() == 0
    sk.close()
    dg.close()


# ------------------------------------------------------------------ sketches

BF_CASES = [("er4096", 256, 1), ("rmat12", 320, 2), ("hub", 128, 3), ("rmat10", 2048, 1), ("rmat10", 64, 1),
            ("k40", 1024, 2), ("rmat_n1000", 576, 1), ("isolated", 256, 1), ("single_edge", 128, 2)]


def _bf_pair(ctx, name, B, b, seed=7):
    g, dg = dgraph(ctx, name)
    say(f"bf build {name} B={B} b={b}")
    sk = dg.build_sketches("bf", B, b, seed=seed)
    ref = oracle.build_sketches(g, oracle.KIND_BF, B, b, seed=seed)
    return g, dg, sk, ref


@pytest.mark.parametrize("name,B,b", BF_CASES)
def test_bf_build_bitexact(ctx, name, B, b):
    g, dg, sk, ref = _bf_pair(ctx, name, B, b)
    rows, pc = sk.export()
    torch.cuda.synchronize()
    assert np.array_equal(np_(rows), ref.words.view(np.uint8).reshape(g.n, B // 8))
    assert np.array_equal(np_(pc).astype(np.uint32), ref.pc)
    sk.close()
    dg.close()


KH_CASES = [("rmat12", 32), ("hub", 7), ("er4096", 64), ("k40", 1), ("rmat10", 100), ("isolated", 16)]


@pytest.mark.parametrize("name,k", KH_CASES)
def test_khash_build_bitexact(ctx, name, k):
    g, dg = dgraph(ctx, name)
    say(f"k-hash build {name} k={k}")
    sk = dg.build_sketches("kh", k, seed=5)
    ref = oracle.build_sketches(g, oracle.KIND_KH, k, seed=5)
    rows, _ = sk.export()
    torch.cuda.synchronize()
    assert np.array_equal(np_(rows), ref.sig.view(np.uint8).reshape(g.n, 4 * k))
    sk.close()
    dg.close()


# k = 600 on the hub (degree 5999): no LDS candidates above k = 512, radix select over all elements;
# the big star's hub (degree 199,999): the first top-byte bin exceeds 512 keys, the second fits
OH_CASES = [("rmat12", 32), ("hub", 64), ("er4096", 8), ("k40", 100), ("rmat10", 1), ("wheel7", 3), ("isolated", 4),
            ("hub", 600), ("bigstar", 32)]


@pytest.mark.parametrize("name,k", OH_CASES)
def test_onehash_build_bitexact(ctx, name, k):
    g, dg = dgraph(ctx, name)
    say(f"1-hash build {name} k={k}")
    sk = dg.build_sketches("1h", k, seed=9)
    ref = oracle.build_sketches(g, oracle.KIND_1H, k, seed=9)
    rows, _ = sk.export()
    torch.cuda.synchronize()
    assert np.array_equal(np_(rows), ref.sig.view(np.uint8).reshape(g.n, 4 * k))
    sk.close()
    dg.close()


# ------------------------------------------------------------------ estimates

def _oracle_raw(ref, est, u, v):
    c = ref.counts(u, v)
    if ref.kind == oracle.KIND_BF:
        return c[1] if est == "or" else c[0]
    if ref.kind == oracle.KIND_KH:
        return c
    return c[2] if est == "1h_lit" else c[0]


EST_CASES = [
    ("er4096", "bf", 256, 1, ("and", "l", "or", "pap")),
    ("rmat12", "bf", 320, 2, ("and", "l", "or", "pap")),
    ("hub", "bf", 1024, 1, ("and", "or")),
    ("rmat10", "bf", 2048, 2, ("and", "pap")),
    ("rmat12", "kh", 32, 1, ("kh",)),
    ("hub", "kh", 20, 1, ("kh",)),
    ("hub", "kh", 16, 1, ("kh",)),
    ("er4096", "kh", 64, 1, ("kh",)),
    ("rmat12", "1h", 32, 1, ("1h", "1h_lit")),
    ("er4096", "1h", 64, 1, ("1h", "1h_lit")),
    ("hub", "1h", 16, 1, ("1h", "1h_lit")),
    ("rmat12", "1h", 128, 1, ("1h", "1h_lit")),
    ("rmat12", "1h", 48, 1, ("1h", "1h_lit")),  # lanes 48..63 hold no slot of the rows
    ("hub", "1h", 7, 1, ("1h", "1h_lit")),      # half waves, rows of 7 slots
]
KIND_OF = {"bf": oracle.KIND_BF, "kh": oracle.KIND_KH, "1h": oracle.KIND_1H}


@pytest.mark.parametrize("name,kind,size,b,ests", EST_CASES)
def test_estimates_match_oracle(ctx, name, kind, size, b, ests):
    g, dg = dgraph(ctx, name)
    say(f"estimates {name} {kind} size={size} b={b}")
    sk = dg.build_sketches(kind, size, b, seed=11)
    ref = oracle.build_sketches(g, KIND_OF[kind], size, b, seed=11)
    eu, ev = oracle.upper_edges(g)
    ru, rv = _rand_pairs(g, 3000, seed=size)
    dev = torch.device("cuda", 0)
    tu, tv = torch.from_numpy(ru).to(dev), torch.from_numpy(rv).to(dev)
    for est in ests:
        say(f"  estimator {est}")
        # all upper edges (u = v = NULL)
        e_gpu, r_gpu = sk.intersect(est)
        torch.cuda.synchronize()
        assert np.array_equal(np_(r_gpu).astype(np.uint32), _oracle_raw(ref, est, eu, ev))
        _close(np_(e_gpu), ref.estimate(eu, ev, est))
        # explicit pairs, including non-adjacent and u == v
        e2, r2 = sk.intersect(est, tu, tv)
        torch.cuda.synchronize()
        assert np.array_equal(np_(r2).astype(np.uint32), _oracle_raw(ref, est, ru, rv))
        _close(np_(e2), ref.estimate(ru, rv, est))
        # triangle count
        tc = sk.tc(est)
        _close([tc], [oracle.tc(ref, est)], rtol=1e-9)
        # clustering coefficient and transitivity
        cc, trans = sk.cc(est, transitivity=True)
        torch.cuda.synchronize()
        want_cc = oracle.cc(ref, est)
        _close32(np_(cc), want_cc)
        wedges = float(np.sum(g.degrees() * (g.degrees() - 1) // 2))
        if wedges:
            _close([trans], [3 * oracle.tc(ref, est) / wedges], rtol=1e-9)
        # Jaccard on edges and on pairs
        j = sk.jaccard(est)
        j2 = sk.jaccard(est, tu, tv)
        torch.cuda.synchronize()
        _close32(np_(j), oracle.jaccard(ref, est, eu, ev))
        _close32(np_(j2), oracle.jaccard(ref, est, ru, rv))
    sk.close()
    dg.close()


def test_estimator_kind_mismatch_is_rejected(ctx):
    g, dg = dgraph(ctx, "wheel7")
    sk = dg.build_sketches("bf", 128, 1, seed=1)
    with pytest.raises(pg.PGError) as ei:
        sk.tc("kh")
    assert ei.value.code == pg.PG_E_INVALID
    with pytest.raises(pg.PGError):
        dg.close()  # sketches still alive
    sk.close()
    dg.close()


def test_out_of_range_pairs_give_nan_not_a_fault(ctx):
    g, dg = dgraph(ctx, "wheel7")
    sk = dg.build_sketches("bf", 128, 1, seed=1)
    dev = torch.device("cuda", 0)
    u = torch.tensor([0, -1, 3, 8], dtype=torch.int32, device=dev)
    v = torch.tensor([1, 2, 1000, 2], dtype=torch.int32, device=dev)
    est, raw = sk.intersect("and", u, v)
    torch.cuda.synchronize()
    e = np_(est)
    assert np.isfinite(e[0]) and np.all(np.isnan(e[1:]))
    assert np.all(np_(raw)[1:] == -1)
    sk.close()
    dg.close()


def test_zero_pairs(ctx):
    g, dg = dgraph(ctx, "wheel7")
    sk = dg.build_sketches("kh", 8, seed=1)
    dev = torch.device("cuda", 0)
    z = torch.zeros(0, dtype=torch.int32, device=dev)
    est, raw = sk.intersect("kh", z, z)
    assert est.shape[0] == 0 and raw.shape[0] == 0
    assert sk.jaccard("kh", z, z).shape[0] == 0
    sk.close()
    dg.close()


# ------------------------------------------------------------------ exact baseline

@pytest.mark.parametrize("name", ["er4096", "rmat12", "hub", "k40", "wheel7", "isolated", "single_edge"])
def test_exact_baseline(ctx, name):
    g, dg = dgraph(ctx, name)
    say(f"exact {name}")
    eu, ev = oracle.upper_edges(g)
    got = dg.exact_intersect()
    torch.cuda.synchronize()
    assert np.array_equal(np_(got).astype(np.uint32), oracle.exact_pairs(g, eu, ev))
    ru, rv = _rand_pairs(g, 2000, seed=3)
    dev = torch.device("cuda", 0)
    got2 = dg.exact_intersect(torch.from_numpy(ru).to(dev), torch.from_numpy(rv).to(dev))
    torch.cuda.synchronize()
    assert np.array_equal(np_(got2).astype(np.uint32), oracle.exact_pairs(g, ru, rv))
    tc = oracle.exact_tc(g)
    assert dg.exact_tc() == tc
    cc, trans = dg.exact_cc(transitivity=True)
    torch.cuda.synchronize()
    _close32(np_(cc), oracle.exact_cc(g))
    wedges = float(np.sum(g.degrees() * (g.degrees() - 1) // 2))
    if wedges:
        _close([trans], [3 * tc / wedges], rtol=1e-12)
    j = dg.exact_jaccard()
    torch.cuda.synchronize()
    _close32(np_(j), oracle.exact_jaccard(g, eu, ev))
    dg.close()


@pytest.mark.parametrize("name", ["er4096", "rmat12", "hub", "k40", "wheel7", "isolated", "single_edge"])
def test_exact_bitmap(ctx, name):
    """The bitmap intersection: every upper edge and the triangle count, bit-exact."""
    g, dg = dgraph(ctx, name)
    say(f"exact bitmap {name}")
    eu, ev = oracle.upper_edges(g)
    got = dg.exact_intersect(algo=pg.PG_EXACT_BITMAP)
    torch.cuda.synchronize()
    assert np.array_equal(np_(got).astype(np.uint32), oracle.exact_pairs(g, eu, ev))
    assert dg.exact_tc(algo=pg.PG_EXACT_BITMAP) == oracle.exact_tc(g)
    if g.n > 1:  # explicit pair lists are the merge kernel's
        dev = torch.device("cuda", 0)
        t = torch.zeros(1, dtype=torch.int32, device=dev)
        with pytest.raises(pg.PGError) as ei:
            dg.exact_intersect(t, t, algo=pg.PG_EXACT_BITMAP)
        assert ei.value.code == pg.PG_E_UNSUPPORTED
    dg.close()


def test_exact_bitmap_several_windows(ctx):
    """IDs beyond 2^20 take several bitmap windows: a sparse G(n, p) with n = 2^20 + 3000
    (uniform IDs, so most lists span both windows) plus a star and a clique."""
    n = (1 << 20) + 3000
    base = pggen.er(n, 6, seed=9)
    hubs = pggen.disjoint_union(pggen.star(4000), pggen.complete(60))
    g = pggen.disjoint_union(base, hubs)
    say(f"exact bitmap, several windows: n={g.n} nnz={g.nnz}")
    dg = pg.Graph(ctx, g.offsets, g.adj)
    eu, ev = oracle.upper_edges(g)
    got = dg.exact_intersect(algo=pg.PG_EXACT_BITMAP)
    torch.cuda.synchronize()
    assert np.array_equal(np_(got).astype(np.uint32), oracle.exact_pairs(g, eu, ev))
    tc = oracle.exact_tc(g)
    assert dg.exact_tc(algo=pg.PG_EXACT_BITMAP) == tc
    assert dg.exact_tc() == tc
    dg.close()


def test_closed_forms_on_gpu(ctx):
    for n in (5, 33):
        g = pggen.complete(n)
        dg = pg.Graph(ctx, g.offsets, g.adj)
        say(f"closed form K{n}")
        assert dg.exact_tc() == math.comb(n, 3)
        sk = dg.build_sketches("1h", 64, seed=2)  # k >= |N_u u N_v| = n: exact
        assert sk.tc("1h") == pytest.approx(math.comb(n, 3), rel=1e-12)
        sk.close()
        dg.close()
    g = pggen.complete_bipartite(3, 7)
    dg = pg.Graph(ctx, g.offsets, g.adj)
    sk = dg.build_sketches("kh", 32, seed=2)
    assert sk.tc("kh") == 0.0 and dg.exact_tc() == 0
    sk.close()
    dg.close()


# ------------------------------------------------------------------ determinism

def test_bitwise_reproducible(ctx):
    g, dg = dgraph(ctx, "rmat12")
    a = dg.build_sketches("bf", 320, 2, seed=3)
    b = dg.build_sketches("bf", 320, 2, seed=3)
    c = dg.build_sketches("bf", 320, 2, seed=4)
    ra, _ = a.export()
    rb, _ = b.export()
    rc, _ = c.export()
    torch.cuda.synchronize()
    assert torch.equal(ra, rb) and not torch.equal(ra, rc)
    t1, t2 = a.tc("and"), a.tc("and")
    assert t1 == t2 and t1 == b.tc("and")
    cc1, cc2 = a.cc("and"), a.cc("and")
    assert torch.equal(cc1, cc2)
    for s in (a, b, c):
        s.close()
    dg.close()


# ------------------------------------------------------------------ full size

@pytest.fixture(scope="module")
def g20():
    say("generating R-MAT scale 20, edge factor 16")
    return pggen.rmat(20, 16, seed=1)


def test_full_size_rmat20_bf_tc_and_samples(ctx, g20):
    g = g20
    dg = pg.Graph(ctx, g.offsets, g.adj)
    B = dg.bits_for_budget(0.33)
    assert B == oracle.bits_for_budget(g, 0.33)
    eu, ev = oracle.upper_edges(g)
    assert dg.m == eu.shape[0]
    rng = np.random.default_rng(20)
    sample = np.unique(np.concatenate([rng.integers(0, g.n, 3000), np.argsort(-g.degrees())[:50]]))
    for b in (1, 2):
        say(f"full size bf B={B} b={b}")
        sk = dg.build_sketches("bf", B, b, seed=1)
        ref = oracle.build_sketches(g, oracle.KIND_BF, B, b, seed=1)
        rows, pc = sk.export()
        torch.cuda.synchronize()
        rows_np = np_(rows)
        assert np.array_equal(rows_np[sample], ref.words.view(np.uint8).reshape(g.n, B // 8)[sample])
        assert np.array_equal(rows_np, ref.words.view(np.uint8).reshape(g.n, B // 8))
        assert np.array_equal(np_(pc).astype(np.uint32), ref.pc)
        # every edge count, and the triangle-count estimate
        _, raw = sk.intersect("and", want_est=False)
        torch.cuda.synchronize()
        assert np.array_equal(np_(raw).astype(np.uint32), ref.counts(eu, ev)[0])
        _close([sk.tc("and")], [oracle.tc(ref, "and")], rtol=1e-9)
        cc = sk.cc("and")
        torch.cuda.synchronize()
        _close32(np_(cc)[sample], oracle.local_cc_from_arc_values(g, ref.estimate(*oracle.arcs(g), "and"))[sample])
        sk.close()
    dg.close()


def test_full_size_rmat20_khash_and_exact(ctx, g20):
    g = g20
    dg = pg.Graph(ctx, g.offsets, g.adj)
    say("full size k-hash k=32")
    sk = dg.build_sketches("kh", 32, seed=1)
    ref = oracle.build_sketches(g, oracle.KIND_KH, 32, seed=1)
    rows, _ = sk.export()
    torch.cuda.synchronize()
    assert np.array_equal(np_(rows), ref.sig.view(np.uint8).reshape(g.n, 128))
    _close([sk.tc("kh")], [oracle.tc(ref, "kh")], rtol=1e-9)
    sk.close()
    say("full size exact triangle count")
    assert dg.exact_tc() == oracle.exact_tc_listing(g)
    # sampled exact intersections (hub edges included)
    eu, ev = oracle.upper_edges(g)
    rng = np.random.default_rng(21)
    idx = np.concatenate([rng.integers(0, eu.shape[0], 4000), np.arange(200)])
    got = dg.exact_intersect()
    torch.cuda.synchronize()
    assert np.array_equal(np_(got).astype(np.uint32)[idx], oracle.exact_pairs(g, eu[idx], ev[idx]))
    dg.close()


def test_estimators_on_two_streams_do_not_interfere(ctx):
    """Every Bloom-filter estimator has its own table, filled when the set is
    made: AND, OR, limit and the existing estimator interleaved on two streams
    without waits give exactly what each gives alone."""
    g = graph("rmat12")
    say("two streams alternating Bloom-filter estimators, rmat12 bf320")
    dg = pg.Graph(ctx, g.offsets, g.adj)
    sk = dg.build_sketches("bf", 320, 1, seed=3)
    ests = ["and", "or", "l", "pap"]
    tc_alone = {e: sk.tc(e) for e in ests}
    edge_alone = {e: sk.intersect(e, want_raw=False)[0].clone() for e in ests}
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    rounds = 6
    tcs = torch.full((rounds * len(ests),), float("nan"), dtype=torch.float64, device="cuda")
    edges = [torch.full((dg.m,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(rounds * len(ests))]
    torch.cuda.synchronize()
    for i in range(rounds * len(ests)):
        e, st = ests[i % len(ests)], streams[i % 2]
        sk.tc_async(e, tcs[i:i + 1], stream=st)
        pg.pg_intersect_edges(ctx.h, sk.h, pg.ESTIMATORS[e], None, None, 0, edges[i], None, st)
    torch.cuda.synchronize()
    for i in range(rounds * len(ests)):
        e = ests[i % len(ests)]
        assert tcs[i].item() == tc_alone[e], (i, e)
        assert torch.equal(edges[i], edge_alone[e]), (i, e)
    sk.close()
    dg.close()


@pytest.mark.parametrize("nbytes", [16, 4096, 16 * 1023, 16 * (256 * 4 * 3 + 77), 1 << 24])
def test_reference_copy_kernel(ctx, nbytes):
    """pg_copy (the stream-copy reference for bandwidth and byte counters) copies
    every byte: whole tiles and the ragged tail."""
    say(f"pg_copy {nbytes} bytes")
    g = torch.Generator().manual_seed(nbytes)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, generator=g).cuda()
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
    pg.pg_copy(ctx.h, dst[:nbytes], src, nbytes)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src)
    assert int(dst[nbytes:].sum()) == 0  # nothing written past the end


def test_cc_over_slabs_every_vertex(ctx):
    """The clustering coefficient over XCD slabs of all of N_v: a 40,000-leaf
    star (its items in every slab exceed the 2,048-arc chunk, so they run as
    heavy chunks), an R-MAT graph (light and medium items, whole vertices) and
    isolated vertices; every vertex against the oracle, for Bloom filters with
    a ratio estimator (AND) and one that reads the popcounts (OR), and for
    k-hash signatures, and the transitivity. The same graph also checks every
    vertex's 1-hash coefficient (the vertex plan with heavy chunks; half waves
    at k = 16, the ID table at k = 64, the key search at k = 100, and a KMV
    estimator)."""
    g = pggen.disjoint_union(pggen.star(40000), pggen.rmat(12, 16, seed=5), pggen.er(50, 0, seed=1))
    say(f"cc over slabs: n={g.n}")
    dg = pg.Graph(ctx, g.offsets, g.adj, validate=True)
    sk = dg.build_sketches("bf", 512, 1, seed=2)
    ref = oracle.build_sketches(g, oracle.KIND_BF, 512, 1, seed=2)
    for est in ("and", "or"):
        cc, trans = sk.cc(est, transitivity=True)
        torch.cuda.synchronize()
        _close32(np_(cc), oracle.cc(ref, est))
        wedges = float(np.sum(g.degrees() * (g.degrees() - 1) // 2))
        _close([trans], [3 * oracle.tc(ref, est) / wedges], rtol=1e-9)
        again = sk.cc(est)
        assert torch.equal(cc, again)  # the same bits on a second call
    sk.close()
    for k in (16, 32, 64):  # k-hash over the same plan
        say(f"cc over slabs: k-hash k={k}")
        sk = dg.build_sketches("kh", k, seed=4)
        ref = oracle.build_sketches(g, oracle.KIND_KH, k, seed=4)
        cc, trans = sk.cc("kh", transitivity=True)
        torch.cuda.synchronize()
        _close32(np_(cc), oracle.cc(ref, "kh"))
        _close([trans], [3 * oracle.tc(ref, "kh") / wedges], rtol=1e-9)
        sk.close()
    for k, ests in ((16, ("1h", "1h_lit")), (64, ("1h", "1h_lit", "kmv")), (100, ("1h",))):
        say(f"cc over slabs: 1-hash k={k}")
        sk = dg.build_sketches("1h", k, seed=6)
        ref = oracle.build_sketches(g, oracle.KIND_1H, k, seed=6)
        for est in ests:
            cc, trans = sk.cc(est, transitivity=True)
            torch.cuda.synchronize()
            _close32(np_(cc), oracle.cc(ref, est))
            _close([trans], [3 * oracle.tc(ref, est) / wedges], rtol=1e-9)
        sk.close()
    dg.close()


def _id_bucket8(x):
    """Top 8 bits of x * 0x9E3779B1 mod 2^32: the bucket of vertex ID x in the
    ID table the 1-hash ratio kernels build in LDS for 64 < k <= 128 (256
    buckets); its top 7 bits are the bucket for k <= 64 (128 buckets)."""
    return ((x * 0x9E3779B1) & 0xFFFFFFFF) >> 24


def test_onehash_id_table_full_buckets(ctx):
    """1-hash triangle count and clustering coefficient where an owner's IDs
    all fall in one bucket of the kernels' ID table: hub 0 has 160 neighbours
    from the first bucket (its kept IDs fill a run of buckets, so lookups walk
    past full buckets), hub 2 has 150 from the last bucket (the chain wraps to
    the first); the hubs' neighbours form paths and share hub 1, and random
    edges join the rest. TC and every vertex's CC against the oracle, two
    elements per lane (k = 128), whole waves (k = 64) and half waves (k = 32),
    both ratio readings."""
    n = 60000
    b0 = [x for x in range(3, n) if _id_bucket8(x) == 0][:160]
    blast = [x for x in range(3, n) if _id_bucket8(x) == 255][:150]
    assert len(b0) == 160 and len(blast) == 150
    src, dst = [0], [1]
    for hub, ids in ((0, b0), (2, blast)):
        src += [hub] * len(ids) + ids[:-1] + [1] * len(ids)
        dst += ids + ids[1:] + ids
    rng = np.random.default_rng(5)
    src = np.concatenate([np.array(src), rng.integers(0, n, 20000)])
    dst = np.concatenate([np.array(dst), rng.integers(0, n, 20000)])
    g = pggen.from_pairs(n, src, dst)
    say(f"ID-table buckets: n={g.n} nnz={g.nnz}")
    dg = pg.Graph(ctx, g.offsets, g.adj, validate=True)
    wedges = float(np.sum(g.degrees() * (g.degrees() - 1) // 2))
    for k in (128, 64, 32):
        sk = dg.build_sketches("1h", k, seed=7)
        ref = oracle.build_sketches(g, oracle.KIND_1H, k, seed=7)
        for est in ("1h", "1h_lit"):
            say(f"  k={k} {est}")
            _close([sk.tc(est)], [oracle.tc(ref, est)], rtol=1e-9)
            cc, trans = sk.cc(est, transitivity=True)
            torch.cuda.synchronize()
            _close32(np_(cc), oracle.cc(ref, est))
            _close([trans], [3 * oracle.tc(ref, est) / wedges], rtol=1e-9)
        sk.close()
    dg.close()


@pytest.mark.parametrize("bits", [64, 320, 1024])
def test_all_edges_over_slabs_equal_explicit_pairs(ctx, bits):
    """The all-edges calls (no pairs given) walk the triangle count's slab
    plan and write each edge at its CSR position; their estimates, raw counts
    and similarities equal, bit for bit, the pair kernel's on the same edges
    passed explicitly, for every Bloom-filter estimator, on a graph with
    heavy chunks (a 40,000-leaf star), sliced and whole vertices."""
    g = pggen.disjoint_union(pggen.star(40000), pggen.rmat(12, 16, seed=6))
    say(f"all edges over slabs, B={bits}")
    dg = pg.Graph(ctx, g.offsets, g.adj, validate=True)
    sk = dg.build_sketches("bf", bits, 2, seed=3)
    eu, ev = dg.upper_edges()
    eu, ev = eu.clone(), ev.clone()  # other buffers: the pair kernel's path
    ref = oracle.build_sketches(g, oracle.KIND_BF, bits, 2, seed=3)
    ou, ov = oracle.upper_edges(g)
    assert np.array_equal(np_(eu), ou) and np.array_equal(np_(ev), ov)
    for est in ("and", "l", "or", "pap"):
        e_all, r_all = sk.intersect(est)
        e_lst, r_lst = sk.intersect(est, eu, ev)
        torch.cuda.synchronize()
        assert torch.equal(r_all, r_lst), est
        assert np.array_equal(np_(e_all).view(np.uint64), np_(e_lst).view(np.uint64)), est
        assert np.array_equal(np_(r_all).astype(np.uint32), _oracle_raw(ref, est, ou, ov)), est
        for measure in ("cn", "jaccard", "overlap", "total"):
            s_all = sk.similarity(est, measure)
            s_lst = sk.similarity(est, measure, eu, ev)
            torch.cuda.synchronize()
            assert np.array_equal(np_(s_all).view(np.uint32), np_(s_lst).view(np.uint32)), (est, measure)
    _close32(np_(sk.jaccard("and")), oracle.jaccard(ref, "and", ou, ov))
    sk.close()
    dg.close()
