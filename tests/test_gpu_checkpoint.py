"""Checkpoint / resume of sketch sets through the C ABI (pg_sketches_export,
pg_sketches_import) and the binding's save / load: an imported set is
bit-identical to the exported one (rows, popcounts), gives bit-identical
estimates and triangle counts, rebuilds to the same rows from its seed, and
matches the oracle's rows."""
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


CASES = [  # (kind, size, b, oriented, estimator)
    ("bf", 320, 1, False, "and"),
    ("bf", 2048, 2, False, "or"),
    ("bf", 256, 1, True, "and"),
    ("kh", 32, 1, False, "kh"),
    ("1h", 64, 1, False, "1h"),
    ("1h", 16, 1, True, "kmv"),
]
KIND_OF = {"bf": oracle.KIND_BF, "kh": oracle.KIND_KH, "1h": oracle.KIND_1H}


@pytest.fixture(scope="module")
def graph(ctx):
    g = pggen.rmat(12, 16, seed=3)
    dg = pg.Graph(ctx, g.offsets, g.adj)
    yield g, dg
    dg.close()


def np_(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("kind,size,b,oriented,est", CASES)
def test_export_import_round_trip(graph, kind, size, b, oriented, est):
    g, dg = graph
    say(f"checkpoint {kind} size={size} b={b} oriented={oriented}")
    sk = dg.build_sketches(kind, size, b, seed=17, oriented=oriented)
    rows, pc = sk.export()
    for use_pc in (True, False):
        sk2 = dg.import_sketches(kind, size, b, 17, rows, pc if use_pc else None, oriented=oriented)
        assert sk2.oriented == oriented and sk2.kind == sk.kind and sk2.seed == 17
        rows2, pc2 = sk2.export()
        torch.cuda.synchronize()
        assert torch.equal(rows, rows2)
        if pc is not None:
            assert torch.equal(pc, pc2)
        e1, r1 = sk.intersect(est)
        e2, r2 = sk2.intersect(est)
        torch.cuda.synchronize()
        assert torch.equal(r1, r2) and torch.equal(e1, e2)
        assert sk.tc(est) == sk2.tc(est)
        # the imported set rebuilds from its seed to the same rows
        sk2.rebuild()
        rows3, _ = sk2.export()
        torch.cuda.synchronize()
        assert torch.equal(rows, rows3)
        sk2.close()
    # and the rows are the oracle's
    src = oracle.oriented(g) if oriented else g
    ref = oracle.build_sketches(src, KIND_OF[kind], size, b, seed=17)
    want = ref.words.view(np.uint8) if kind == "bf" else ref.sig.view(np.uint8)
    assert np.array_equal(np_(rows), want.reshape(g.n, -1))
    sk.close()


def test_save_and_load(graph, tmp_path):
    g, dg = graph
    sk = dg.build_sketches("bf", 320, 2, seed=5)
    path = tmp_path / "bf.npz"
    sk.save(path)
    sk2 = dg.load_sketches(path)
    assert (sk2.kind, sk2.size, sk2.b, sk2.seed, sk2.oriented) == (sk.kind, sk.size, sk.b, sk.seed, False)
    assert sk2.tc("and") == sk.tc("and")
    r1, p1 = sk.export()
    r2, p2 = sk2.export()
    torch.cuda.synchronize()
    assert torch.equal(r1, r2) and torch.equal(p1, p2)
    sk2.close()
    sk.close()
    sk = dg.build_sketches("1h", 32, seed=9, oriented=True)
    sk.save(tmp_path / "oh.npz")
    sk2 = dg.load_sketches(tmp_path / "oh.npz")
    assert sk2.oriented and sk2.tc("1h") == sk.tc("1h")
    sk2.close()
    sk.close()


def test_load_refuses_another_graph(ctx, graph, tmp_path):
    g, dg = graph
    sk = dg.build_sketches("kh", 16, seed=2)
    sk.save(tmp_path / "kh.npz")
    sk.close()
    other = pggen.rmat(11, 16, seed=3)
    dg2 = pg.Graph(ctx, other.offsets, other.adj)
    with pytest.raises(ValueError):
        dg2.load_sketches(tmp_path / "kh.npz")
    dg2.close()


def test_import_rejects_bad_parameters(ctx, graph):
    g, dg = graph
    rows = torch.zeros((g.n, 40), dtype=torch.uint8, device="cuda")
    with pytest.raises(pg.PGError):
        dg.import_sketches("bf", 321, 1, 1, rows)  # not a multiple of 64
    lib = pg.load()
    h = pg._vp()
    assert lib.pg_sketches_import(ctx.h, dg.h, pg.PG_BF, 320, 1, 1, None, None, None,
                                  pg.ctypes.byref(h)) == pg.PG_E_INVALID


@pytest.mark.parametrize("oriented", [False, True])
def test_rebuilds_keep_rows_of_empty_sets_zero(ctx, oriented):
    """Builds after the first leave the rows of vertices without neighbours (in
    the sketched lists) untouched, as they are zero under every seed; an import
    can bring other rows, so the build after it writes every row again."""
    g = pggen.disjoint_union(pggen.er(500, 8, seed=2), pggen.from_pairs(300, [], []), pggen.star(40))
    dg = pg.Graph(ctx, g.offsets, g.adj)
    src = oracle.oriented(g) if oriented else g
    empty = np.flatnonzero(np.diff(src.offsets) == 0)
    assert empty.size >= 300
    sk = dg.build_sketches("bf", 320, 1, seed=3, oriented=oriented)
    for seed in (4, 5, 3):  # consecutive rebuilds: every row is the oracle's
        sk.rebuild(seed)
        rows, pc = sk.export()
        torch.cuda.synchronize()
        ref = oracle.build_sketches(src, oracle.KIND_BF, 320, 1, seed=seed)
        assert np.array_equal(np_(rows), ref.words.view(np.uint8).reshape(g.n, -1))
        assert np.array_equal(np_(pc).astype(np.uint32), ref.pc)
    noisy = rows.clone()
    noisy[torch.from_numpy(empty).to(noisy.device)] = 0xA5
    sk2 = dg.import_sketches("bf", 320, 1, 3, noisy, None, oriented=oriented)
    r_noisy, _ = sk2.export()
    assert torch.equal(r_noisy, noisy)
    sk2.rebuild()
    r2, p2 = sk2.export()
    torch.cuda.synchronize()
    assert torch.equal(r2, rows) and torch.equal(p2, pc)
    sk2.close()
    sk.close()
    dg.close()


def test_import_rejects_popcounts_that_differ_from_the_rows(ctx, graph):
    """The OR estimator indexes its table with pc_u + pc_v - c: an import counts
    the ones of the rows itself and refuses given popcounts that differ."""
    g, dg = graph
    say("import with a corrupted popcount")
    sk = dg.build_sketches("bf", 320, 1, seed=5)
    rows, pc = sk.export()
    bad = pc.clone()
    bad[7] += 1000
    with pytest.raises(pg.PGError) as ei:
        dg.import_sketches("bf", 320, 1, 5, rows, bad)
    assert ei.value.code == pg.PG_E_INVALID
    sk2 = dg.import_sketches("bf", 320, 1, 5, rows, pc)  # the true counts are accepted
    assert sk2.tc("or") == sk.tc("or")
    sk2.close()
    sk.close()


def test_load_refuses_a_graph_of_the_same_size(ctx, graph, tmp_path):
    """Same n and m, other edges: the CSR fingerprint in the file differs."""
    g, dg = graph
    sk = dg.build_sketches("bf", 256, 1, seed=2)
    sk.save(tmp_path / "bf.npz")
    sk.close()
    perm = np.random.default_rng(1).permutation(g.n).astype(np.int32)  # relabelled copy: same n and m
    eu, ev = oracle.upper_edges(g)
    other = pggen.from_pairs(g.n, perm[eu], perm[ev])
    assert other.n == g.n and other.nnz == g.nnz and not np.array_equal(other.adj, g.adj)
    dg2 = pg.Graph(ctx, other.offsets, other.adj)
    with pytest.raises(ValueError, match="fingerprint"):
        dg2.load_sketches(tmp_path / "bf.npz")
    dg2.close()
