"""Batched small graphs on the GPU: per-graph results match the oracle, do
not depend on the tuning parameters, and HIP-graph replays equal the eager run."""
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
def batch_env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    graphs, _ = pggen.graph_batch(count=24, seed0=11, log2_lo=6.0, log2_hi=11.0)
    # every row width the batch path instantiates, W = 1..16 words (64..1024 bits)
    bits = [64 * (1 + i % 16) for i in range(len(graphs))]
    extra = [pggen.disjoint_union(pggen.star(700), pggen.complete(12)), pggen.from_pairs(5, [], []),
             pggen.from_pairs(1, [], []), pggen.wheel(9)]
    graphs += extra
    bits += [128, 64, 64, 1024]
    assert sorted({B // 64 for B in bits}) == list(range(1, 17))
    say(f"batch of {len(graphs)} graphs, n total {sum(g.n for g in graphs)}")
    ctx = pg.Context(0)
    bt = pg.Batch(ctx, graphs, bits, b=2, seed=5)
    yield graphs, bits, ctx, bt
    bt.close()
    ctx.close()


def _oracle(graphs, bits, b, seed, est):
    tcs, ccs = [], []
    for g, B in zip(graphs, bits):
        ref = oracle.build_sketches(g, oracle.KIND_BF, B, b, seed=seed)
        tcs.append(oracle.tc(ref, est) if g.nnz else 0.0)
        ccs.append(oracle.cc(ref, est))
    return np.array(tcs), np.concatenate(ccs)


@pytest.mark.parametrize("est", ["and", "l", "pap"])
def test_batch_matches_oracle(batch_env, est):
    graphs, bits, ctx, bt = batch_env
    bt.run(est)
    tc, cc = bt.results()
    want_tc, want_cc = _oracle(graphs, bits, 2, 5, est)
    assert np.allclose(tc, want_tc, rtol=1e-9, atol=1e-9)
    assert np.allclose(cc, want_cc, rtol=1e-6 + 2.0**-23, atol=1e-30)


def test_batch_independent_of_tuning(batch_env):
    graphs, bits, ctx, bt = batch_env
    outs = []
    for tile, bpc in [(32, 1), (64, 4), (256, 8), (4096, 2)]:
        say(f"tile {tile} blocks/CU {bpc}")
        bt.set_params(tile, bpc)
        bt.run("and")
        outs.append(bt.results())
    for tc, cc in outs[1:]:
        assert tc.tobytes() == outs[0][0].tobytes() and cc.tobytes() == outs[0][1].tobytes()
    ms = bt.autotune("and")
    assert ms > 0
    tile, bpc = bt.params()
    assert tile % 32 == 0 and bpc >= 1
    bt.run("and")
    tc, cc = bt.results()
    assert tc.tobytes() == outs[0][0].tobytes() and cc.tobytes() == outs[0][1].tobytes()


def test_batch_graph_replays_equal_eager(batch_env):
    graphs, bits, ctx, bt = batch_env
    bt.run("and")
    tc0, cc0 = bt.results()
    s = torch.cuda.Stream()
    bt.capture("and", stream=s)
    for rep in range(3):
        say(f"replay {rep}")
        bt.replay(stream=s)
        tc, cc = bt.results(stream=s)
        assert tc.tobytes() == tc0.tobytes() and cc.tobytes() == cc0.tobytes()
        # eager work between replays (a run with another estimator, then restore)
        bt.run("l")
        torch.cuda.synchronize()
    tc, cc = bt.results()
    want_tc, _ = _oracle(graphs, bits, 2, 5, "l")
    assert np.allclose(tc, want_tc, rtol=1e-9, atol=1e-9)


def test_batch_rejects_bad_graphs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = pg.Context(0)
    bad = pggen.CSR(3, np.array([0, 1, 2, 2], np.int32), np.array([1, 2], np.int32))  # asymmetric
    with pytest.raises(pg.PGError) as ei:
        pg.Batch(ctx, [pggen.cycle(4), bad], [64, 64])
    assert ei.value.code == pg.PG_E_GRAPH
    with pytest.raises(pg.PGError) as ei:
        pg.Batch(ctx, [pggen.cycle(4)], [100])
    assert ei.value.code == pg.PG_E_INVALID
    ctx.close()


@pytest.mark.timeout(600)
def test_full_batch_workload_matches_oracle():
    """The batch the benchmark times (512 graphs, n log-uniform in [2^8, 2^16],
    half G(n, p), half R-MAT; 128..1024-bit filters, so every row width 2..16):
    every graph's triangle count and every vertex's clustering coefficient
    against the oracle, after an eager run and after a HIP-graph replay."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    say("generating the 512-graph batch")
    graphs, bits = pggen.graph_batch(count=512, seed0=1)
    assert sorted({B // 64 for B in bits}) == list(range(2, 17))
    ctx = pg.Context(0)
    bt = pg.Batch(ctx, graphs, bits, b=1, seed=1)
    say("eager run")
    bt.run("and")
    tc, cc = bt.results()
    say("oracle over the 512 graphs")
    want_tc, want_cc = _oracle(graphs, bits, 1, 1, "and")
    assert np.allclose(tc, want_tc, rtol=1e-9, atol=1e-9)
    assert np.allclose(cc, want_cc, rtol=1e-6 + 2.0**-23, atol=1e-30)
    say("captured replay")
    s = torch.cuda.Stream()
    bt.capture("and", stream=s)
    bt.replay(stream=s)
    tc2, cc2 = bt.results(stream=s)
    assert tc2.tobytes() == tc.tobytes() and cc2.tobytes() == cc.tobytes()
    bt.close()
    ctx.close()
