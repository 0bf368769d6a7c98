"""pg_tc_noalloc (the triangle count for callers that cannot allocate) against
pg_tc_async, through the C ABI: the same estimate bit for bit, on two calls in
a row whose second input is smaller, and within 1e-9 of the FP64 oracle.
The entry point shares the library's fixed per-device workspace, so every call
here runs on one stream, in order."""
import sys

import numpy as np
import pytest

import oracle
import pggen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2208_11469_amd as pg  # noqa: E402

RTOL_ORACLE = 1e-9


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


def _oracle_tc(g, kind, size, b, seed, est):
    ref = oracle.build_sketches(g, {"bf": oracle.KIND_BF, "kh": oracle.KIND_KH, "1h": oracle.KIND_1H}[kind], size, b,
                                seed=seed)
    return oracle.tc(ref, est)


# (name, graph, kind, size, b, estimator): the Bloom-filter slab kernel (W = 5
# and 4), the per-edge general path (W = 32), k-hash and 1-hash slab kernels
CASES = [
    ("rmat14_bf320", lambda: pggen.rmat(14, 16, seed=3), "bf", 320, 1, "and"),
    ("er3000_bf256_or", lambda: pggen.er(3000, 12, seed=5), "bf", 256, 1, "or"),
    ("rmat12_bf2048", lambda: pggen.rmat(12, 16, seed=1), "bf", 2048, 2, "and"),
    ("rmat12_kh32", lambda: pggen.rmat(12, 16, seed=2), "kh", 32, 1, "kh"),
    ("er2000_1h32", lambda: pggen.er(2000, 20, seed=7), "1h", 32, 1, "1h"),
]


def _setup(ctx, make, kind, size, b):
    g = make()
    dg = pg.Graph(ctx, g.offsets, g.adj)
    sk = dg.build_sketches(kind, size, b, seed=11)
    return g, dg, sk


def test_noalloc_needs_the_plan(ctx):
    say("noalloc before the plan exists: rmat10 bf256")
    g = pggen.rmat(10, 16, seed=4)
    dg = pg.Graph(ctx, g.offsets, g.adj)
    sk = dg.build_sketches("bf", 256, 1, seed=1)
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    with pytest.raises(pg.PGError) as ei:
        pg.pg_tc_noalloc(ctx.h, sk.h, pg.PG_EST_BF_AND, out)
    assert ei.value.code == pg.PG_E_UNSUPPORTED
    ref = torch.zeros(1, dtype=torch.float64, device="cuda")
    pg.pg_tc_async(ctx.h, sk.h, pg.PG_EST_BF_AND, ref)  # builds the plan
    pg.pg_tc_noalloc(ctx.h, sk.h, pg.PG_EST_BF_AND, out)
    torch.cuda.synchronize()
    assert out.item() == ref.item()
    sk.close()
    dg.close()


@pytest.mark.parametrize("big,small", [(0, 1), (2, 4), (3, 1)])
def test_noalloc_two_calls_in_a_row(ctx, big, small):
    runs = []
    for idx in (big, small):
        name, make, kind, size, b, est = CASES[idx]
        say(f"setup {name}")
        g, dg, sk = _setup(ctx, make, kind, size, b)
        ref = torch.zeros(1, dtype=torch.float64, device="cuda")
        pg.pg_tc_async(ctx.h, sk.h, pg.ESTIMATORS[est], ref)  # the existing entry point (and the plan)
        torch.cuda.synchronize()
        runs.append((name, g, dg, sk, kind, size, b, est, ref))
    outs = []
    for name, g, dg, sk, kind, size, b, est, ref in runs:  # back to back on one stream, no sync between
        say(f"pg_tc_noalloc {name}")
        out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        pg.pg_tc_noalloc(ctx.h, sk.h, pg.ESTIMATORS[est], out)
        outs.append(out)
    torch.cuda.synchronize()
    assert runs[1][1].n < runs[0][1].n or runs[1][1].nnz < runs[0][1].nnz  # the second input is smaller
    for (name, g, dg, sk, kind, size, b, est, ref), out in zip(runs, outs):
        got, want = out.item(), ref.item()
        assert got == want, (name, got, want)
        tc_o = _oracle_tc(g, kind, size, b, 11, est)
        assert abs(got - tc_o) <= RTOL_ORACLE * max(abs(tc_o), 1.0), (name, got, tc_o)
    for name, g, dg, sk, *_ in runs:
        sk.close()
        dg.close()


def test_noalloc_repeated_calls_stay_identical(ctx):
    name, make, kind, size, b, est = CASES[0]
    say(f"repeated pg_tc_noalloc {name}")
    g, dg, sk = _setup(ctx, make, kind, size, b)
    ref = torch.zeros(1, dtype=torch.float64, device="cuda")
    pg.pg_tc_async(ctx.h, sk.h, pg.ESTIMATORS[est], ref)
    outs = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
    for i in range(8):
        pg.pg_tc_noalloc(ctx.h, sk.h, pg.ESTIMATORS[est], outs[i:i + 1])
    torch.cuda.synchronize()
    assert np.all(outs.cpu().numpy() == ref.item())
    sk.close()
    dg.close()
