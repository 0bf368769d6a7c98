"""GPU parity of vertex similarity (Listing "lst:sim"), Jarvis-Patrick
clustering (Listing "lst:cl") and cluster labels, through the C ABI, against
the oracle.

Similarities are FP32 outputs rounded once from FP64: checked at 1e-6 relative
plus one FP32 rounding. The clustering decision (similarity > tau) is taken in
FP64 on both sides; thresholds are placed midway between neighbouring distinct
oracle values, so an FP64 rounding difference cannot move an edge across
them, and then the masks must match bit for bit. Cluster labels are unique
(the smallest vertex ID of each component), so they must match bit for bit.
"""
import sys

import numpy as np
import pytest

import oracle
import pggen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2208_11469_amd as pg  # noqa: E402

RTOL = 1e-6
MEASURES = {"cn": oracle.SIM_COMMON, "jaccard": oracle.SIM_JACCARD, "overlap": oracle.SIM_OVERLAP,
            "total": oracle.SIM_TOTAL}


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


def _two_cliques_and_bridge():
    a, b = np.triu_indices(5, 1)
    return pggen.from_pairs(10, np.concatenate([a, a + 5, [4]]), np.concatenate([b, b + 5, [5]]))


def _long_path(n, seed):
    v = np.arange(n - 1)
    perm = np.random.default_rng(seed).permutation(n)
    return pggen.from_pairs(n, perm[v], perm[v + 1])


GRAPHS = {
    "er4096": lambda: pggen.er(4096, 16, seed=1),
    "rmat12": lambda: pggen.rmat(12, 16, seed=1),
    "rmat14": lambda: pggen.rmat(14, 8, seed=3),
    "hub": lambda: pggen.disjoint_union(pggen.star(6000), pggen.er(2000, 10, seed=3), pggen.complete(30)),
    "k40": lambda: pggen.complete(40),
    "cliques": _two_cliques_and_bridge,
    "path": lambda: _long_path(5000, 5),
    "forest": lambda: pggen.disjoint_union(pggen.star(300), pggen.cycle(7), pggen.wheel(9), pggen.from_pairs(40, [], []),
                                           pggen.friendship(5), pggen.complete(3)),
    "isolated": lambda: pggen.from_pairs(50, [], []),
    "single_edge": lambda: pggen.from_pairs(3, [0], [2]),
}
_CACHE = {}


def graph(name):
    if name not in _CACHE:
        _CACHE[name] = GRAPHS[name]()
    return _CACHE[name]


def dgraph(ctx, name):
    g = graph(name)
    say(f"graph {name} n={g.n} nnz={g.nnz}")
    return g, pg.Graph(ctx, g.offsets, g.adj, validate=True)


def np_(t):
    return t.detach().cpu().numpy()


def _close32(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    assert got.shape == want.shape
    err = np.abs(got - want)
    bad = err > 1e-30 + (RTOL + 2.0**-23) * np.abs(want)
    assert not bad.any(), f"{bad.sum()} mismatches, worst {err.max()} at {np.argmax(err)}"


def _taus(vals, quantiles=(0.2, 0.5, 0.9)):
    """Thresholds: below every value, above every value, and midway between
    neighbouring distinct values at a few quantiles (skipping gaps too small to
    separate FP64 rounding differences)."""
    u = np.unique(np.asarray(vals, dtype=np.float64))
    if u.shape[0] == 0:
        return [0.0]
    taus = [float(u[0]) - 1.0, float(u[-1]) + 1.0]
    for q in quantiles:
        for i in range(min(int(q * (u.shape[0] - 1)), u.shape[0] - 2), u.shape[0] - 1):
            if u[i + 1] - u[i] > 1e-9 * max(1.0, abs(float(u[i]))):
                taus.append(0.5 * float(u[i] + u[i + 1]))
                break
    return taus


# (graph, kind, size, b, estimators)
SIM_CASES = [
    ("er4096", "bf", 256, 1, ["and", "l", "or", "pap"]),
    ("rmat12", "bf", 320, 2, ["and"]),
    ("rmat12", "kh", 32, 1, ["kh"]),
    ("hub", "1h", 32, 1, ["1h", "1h_lit"]),
    ("k40", "bf", 1024, 2, ["and", "or"]),
    ("cliques", "1h", 16, 1, ["1h"]),
    ("isolated", "bf", 256, 1, ["and"]),
    ("single_edge", "kh", 8, 1, ["kh"]),
]
KIND_ID = {"bf": oracle.KIND_BF, "kh": oracle.KIND_KH, "1h": oracle.KIND_1H}


@pytest.mark.parametrize("name,kind,size,b,ests", SIM_CASES)
def test_similarity_and_jarvis_patrick_match_oracle(ctx, name, kind, size, b, ests):
    g, dg = dgraph(ctx, name)
    sk = dg.build_sketches(kind, size, b, seed=5)
    ref = oracle.build_sketches(g, KIND_ID[kind], size, b, seed=5)
    eu, ev = oracle.upper_edges(g)
    for est in ests:
        for mname, m in MEASURES.items():
            say(f"{name} {kind}{size} {est} {mname}")
            want = oracle.similarity(ref, est, eu, ev, m)
            got = sk.similarity(est, mname)
            torch.cuda.synchronize()
            _close32(np_(got), want)
            for tau in _taus(want):
                keep, kept = sk.jarvis_patrick(est, mname, tau)
                torch.cuda.synchronize()
                want_keep = oracle.jarvis_patrick(want, tau)
                assert kept == int(want_keep.sum()), (tau, kept)
                assert np.array_equal(np_(keep), want_keep), tau
    sk.close()
    dg.close()


def test_similarity_explicit_pairs(ctx):
    g, dg = dgraph(ctx, "rmat12")
    sk = dg.build_sketches("bf", 256, 1, seed=2)
    ref = oracle.build_sketches(g, oracle.KIND_BF, 256, 1, seed=2)
    rng = np.random.default_rng(9)
    u = rng.integers(0, g.n, 5000).astype(np.int32)
    v = rng.integers(0, g.n, 5000).astype(np.int32)
    u[:7] = v[:7]
    for mname, m in MEASURES.items():
        got = sk.similarity("and", mname, torch.from_numpy(u).cuda(), torch.from_numpy(v).cuda())
        torch.cuda.synchronize()
        _close32(np_(got), oracle.similarity(ref, "and", u, v, m))
        ex = dg.exact_similarity(mname, torch.from_numpy(u).cuda(), torch.from_numpy(v).cuda())
        torch.cuda.synchronize()
        _close32(np_(ex), oracle.exact_similarity(g, u, v, m))
    # IDs outside [0, n) give NaN and touch nothing
    bu = torch.tensor([0, -1, g.n, 3], dtype=torch.int32, device="cuda")
    bv = torch.tensor([g.n + 5, 2, 1, 2**31 - 1], dtype=torch.int32, device="cuda")
    for mname in MEASURES:
        got = np_(sk.similarity("and", mname, bu, bv))
        assert np.all(np.isnan(got)), mname
    sk.close()
    dg.close()


@pytest.mark.parametrize("name", ["er4096", "rmat12", "hub", "k40", "cliques", "forest", "isolated", "single_edge"])
def test_exact_similarity_and_jarvis_patrick(ctx, name):
    g, dg = dgraph(ctx, name)
    eu, ev = oracle.upper_edges(g)
    for mname, m in MEASURES.items():
        want = oracle.exact_similarity(g, eu, ev, m)
        got = dg.exact_similarity(mname)
        torch.cuda.synchronize()
        _close32(np_(got), want)
        for tau in _taus(want):
            for algo in (pg.PG_EXACT_MERGE, pg.PG_EXACT_BITMAP):
                keep, kept = dg.exact_jarvis_patrick(mname, tau, algo=algo)
                torch.cuda.synchronize()
                want_keep = oracle.jarvis_patrick(want, tau)
                assert kept == int(want_keep.sum()), (mname, tau, algo)
                assert np.array_equal(np_(keep), want_keep), (mname, tau, algo)
    dg.close()


@pytest.mark.parametrize("name", ["er4096", "rmat12", "rmat14", "hub", "k40", "cliques", "path", "forest",
                                  "isolated", "single_edge"])
def test_clusters_match_oracle(ctx, name):
    g, dg = dgraph(ctx, name)
    eu, ev = oracle.upper_edges(g)
    masks = {"all": None, "none": np.zeros(eu.shape[0], np.uint8)}
    rng = np.random.default_rng(3)
    masks["random"] = (rng.random(eu.shape[0]) < 0.6).astype(np.uint8)
    x = oracle.exact_similarity(g, eu, ev, oracle.SIM_COMMON)
    masks["jp_cn"] = oracle.jarvis_patrick(x, 0.5)
    for mname, keep in masks.items():
        say(f"clusters {name} {mname}")
        want = oracle.clusters(g.n, eu, ev, keep)
        dkeep = None if keep is None else torch.from_numpy(keep).cuda()
        lab, count = dg.clusters(dkeep)
        torch.cuda.synchronize()
        assert np.array_equal(np_(lab), want), mname
        assert count == oracle.cluster_count(want), mname
    dg.close()


def test_clusters_of_a_gpu_clustering(ctx):
    """The chain as a user runs it: JP mask on the GPU, then its clusters."""
    g, dg = dgraph(ctx, "cliques")
    keep, kept = dg.exact_jarvis_patrick("cn", 0.5)
    lab, count = dg.clusters(keep)
    torch.cuda.synchronize()
    assert kept == 20 and count == 2
    assert np_(lab).tolist() == [0] * 5 + [5] * 5
    dg.close()


def test_bad_arguments_are_rejected(ctx):
    g, dg = dgraph(ctx, "k40")
    sk = dg.build_sketches("bf", 256, 1, seed=1)
    with pytest.raises(pg.PGError):
        sk.similarity("and", 7)
    with pytest.raises(pg.PGError):
        sk.jarvis_patrick("and", "cn", float("nan"))
    with pytest.raises(pg.PGError):
        sk.jarvis_patrick("kh", "cn", 1.0)  # estimator of another sketch kind
    with pytest.raises(pg.PGError):
        dg.exact_jarvis_patrick("cn", 1.0, algo=9)
    lib = pg.load()
    assert lib.pg_jarvis_patrick(ctx.h, sk.h, pg.PG_EST_BF_AND, 0, 1.0, None, None, None) == pg.PG_E_INVALID
    assert lib.pg_clusters(ctx.h, dg.h, None, None, None, None) == pg.PG_E_INVALID
    sk.close()
    dg.close()


# ------------------------------------------------------------------ full size

@pytest.fixture(scope="module")
def g20():
    say("generating R-MAT scale 20, edge factor 16")
    return pggen.rmat(20, 16, seed=1)


@pytest.mark.timeout(600)
def test_full_size_rmat20_jarvis_patrick_and_clusters(ctx, g20):
    g = g20
    dg = pg.Graph(ctx, g.offsets, g.adj)
    eu, ev = oracle.upper_edges(g)
    B = dg.bits_for_budget(0.33)
    say(f"full size exact JP and clusters, m={eu.shape[0]}")
    x = oracle.exact_similarity(g, eu, ev, oracle.SIM_COMMON)
    want_keep = oracle.jarvis_patrick(x, 2.5)
    keep, kept = dg.exact_jarvis_patrick("cn", 2.5)
    torch.cuda.synchronize()
    assert kept == int(want_keep.sum())
    assert np.array_equal(np_(keep), want_keep)
    want = oracle.clusters(g.n, eu, ev, want_keep)
    lab, count = dg.clusters(keep)
    torch.cuda.synchronize()
    assert np.array_equal(np_(lab), want) and count == oracle.cluster_count(want)
    say(f"full size BF-{B} JP (Jaccard) and clusters")
    sk = dg.build_sketches("bf", B, 1, seed=1)
    ref = oracle.build_sketches(g, oracle.KIND_BF, B, 1, seed=1)
    sim = oracle.similarity(ref, "and", eu, ev, oracle.SIM_JACCARD)
    tau = _taus(sim, quantiles=(0.5,))[-1]
    want_keep = oracle.jarvis_patrick(sim, tau)
    keep, kept = sk.jarvis_patrick("and", "jaccard", tau)
    torch.cuda.synchronize()
    assert kept == int(want_keep.sum())
    assert np.array_equal(np_(keep), want_keep)
    want = oracle.clusters(g.n, eu, ev, want_keep)
    lab, count = dg.clusters(keep)
    torch.cuda.synchronize()
    assert np.array_equal(np_(lab), want) and count == oracle.cluster_count(want)
    sk.close()
    dg.close()
