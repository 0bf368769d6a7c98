"""Serving engine on the GPU: continuous batching keeps per-pair results
bit-identical alone and in a mix; admission and validation behave."""
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
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    say("serving env: rmat12, BF 512 b=1, k-hash 32, 1-hash 16")
    g = pggen.rmat(12, 16, seed=7)
    ctx = pg.Context(0)
    dg = pg.Graph(ctx, g.offsets, g.adj, validate=True)
    sks = [dg.build_sketches("bf", 512, 1, seed=3), dg.build_sketches("kh", 32, seed=3),
           dg.build_sketches("1h", 16, seed=3)]
    yield g, ctx, dg, sks
    for s in sks:
        s.close()
    dg.close()
    ctx.close()


KINDS = [(0, "and"), (0, "or"), (0, "l"), (0, "pap"), (1, "kh"), (2, "1h"), (2, "1h_lit")]


def _requests(g, count, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        L = int(2 ** rng.uniform(0, 12))
        u = rng.integers(0, g.n, L).astype(np.int32)
        v = rng.integers(0, g.n, L).astype(np.int32)
        sk, est = KINDS[i % len(KINDS)]
        op = pg.PG_OP_CN if rng.integers(0, 2) == 0 else pg.PG_OP_JACCARD
        reqs.append((op, sk, est, u, v))
    return reqs


def test_alone_equals_mixed_and_matches_direct_calls(env):
    g, ctx, dg, sks = env
    reqs = _requests(g, 40, seed=1)
    srv = pg.Server(dg, sks, max_batches_in_flight=3)
    alone = []
    for op, sk, est, u, v in reqs:
        t, out = srv.submit(op, sk, est, u, v)
        srv.wait(t)
        alone.append(out.copy())
    srv.close()
    say("replaying the mix back to back on one batch slot")
    srv = pg.Server(dg, sks, max_batches_in_flight=1)
    mix = [srv.make_request(op, sk, est, u, v) for op, sk, est, u, v in reqs]
    srv.replay(mix, max_outstanding=len(mix))
    st = srv.stats()
    assert st["completed"] == 40 and st["rejected_invalid"] == 0
    assert st["batches"] < 40, st  # requests that queued behind a running batch were merged
    tickets = [(None, keep[2]) for _, keep in mix]
    dev = torch.device("cuda", 0)
    refs = {0: oracle.build_sketches(g, oracle.KIND_BF, 512, 1, seed=3),
            1: oracle.build_sketches(g, oracle.KIND_KH, 32, seed=3),
            2: oracle.build_sketches(g, oracle.KIND_1H, 16, seed=3)}
    for (op, sk, est, u, v), a, (_, m) in zip(reqs, alone, tickets):
        assert a.tobytes() == m.tobytes()  # bitwise: alone == in the mix
        tu, tv = torch.from_numpy(u).to(dev), torch.from_numpy(v).to(dev)
        if op == pg.PG_OP_CN:
            direct, _ = sks[sk].intersect(est, tu, tv)
            want = refs[sk].estimate(u, v, est)
        else:
            direct = sks[sk].jaccard(est, tu, tv)
            want = oracle.jaccard(refs[sk], est, u, v)
        torch.cuda.synchronize()
        assert direct.cpu().numpy().tobytes() == a.tobytes()
        assert np.allclose(a, want, rtol=1e-6 + (2.0**-23 if op == pg.PG_OP_JACCARD else 0), atol=1e-12)
    srv.close()


def test_admission_by_memory_budget(env):
    g, ctx, dg, sks = env
    srv = pg.Server(dg, sks, memory_budget_bytes=16 * 1000)
    u = np.arange(1000, dtype=np.int32) % g.n
    t1, _ = srv.submit(pg.PG_OP_CN, 0, "and", u, u[::-1].copy())
    with pytest.raises(pg.PGError) as ei:
        srv.submit(pg.PG_OP_CN, 0, "and", u[:10], u[:10])
    assert ei.value.code == pg.PG_E_BUSY
    srv.wait(t1)  # collecting releases the budget
    t2, _ = srv.submit(pg.PG_OP_CN, 0, "and", u[:10], u[:10])
    srv.wait(t2)
    assert srv.stats()["rejected_busy"] == 1
    srv.close()


def test_budget_ranges_split_and_merge(env):
    """The budget is handed out as contiguous ranges of 16-byte pair slots:
    freed neighbours merge, and a request needs one range that holds it."""
    g, ctx, dg, sks = env
    srv = pg.Server(dg, sks, memory_budget_bytes=16 * 1000)
    u = (np.arange(100, dtype=np.int32) * 7) % g.n
    held = [srv.submit(pg.PG_OP_CN, 0, "and", u, u[::-1].copy()) for _ in range(10)]  # the whole budget
    for i in (2, 5):  # two separate holes of 100 pairs
        srv.wait(held[i][0])
    big = np.zeros(150, np.int32)
    with pytest.raises(pg.PGError) as ei:
        srv.submit(pg.PG_OP_CN, 0, "and", big, big)
    assert ei.value.code == pg.PG_E_BUSY
    srv.wait(held[3][0])  # merges with the hole before it: 200 pairs in one range
    t, out = srv.submit(pg.PG_OP_CN, 0, "and", big, big)
    t2, out2 = srv.submit(pg.PG_OP_CN, 0, "and", u[:100], u[:100])  # the other hole, exactly
    # 50 pairs are left, at the end of the merged range
    with pytest.raises(pg.PGError) as ei:
        srv.submit(pg.PG_OP_CN, 0, "and", u[:60], u[:60])
    assert ei.value.code == pg.PG_E_BUSY
    for i in (0, 1, 4, 6, 7, 8, 9):
        srv.wait(held[i][0])
    srv.wait(t)
    srv.wait(t2)
    t3, _ = srv.submit(pg.PG_OP_CN, 0, "and", np.zeros(1000, np.int32), np.zeros(1000, np.int32))  # all merged
    srv.wait(t3)
    ref = pg.Server(dg, sks)
    tr, want = ref.submit(pg.PG_OP_CN, 0, "and", u, u[::-1].copy())
    ref.wait(tr)
    for _, o in held:
        assert o.tobytes() == want.tobytes()
    ref.close()
    srv.close()


def test_budget_split_into_parts(env):
    """With a budget of many largest requests the arena is split into 16 parts:
    one thread's requests fill its home part and then the others, the whole
    budget is admitted, one more pair is not, and collecting returns every
    range (the same fill succeeds again)."""
    g, ctx, dg, sks = env
    srv = pg.Server(dg, sks, max_pairs_per_request=64, memory_budget_bytes=16 * 4096)  # 16 parts of 256 pairs
    rng = np.random.default_rng(21)
    u = rng.integers(0, g.n, 64).astype(np.int32)
    v = rng.integers(0, g.n, 64).astype(np.int32)
    ref = pg.Server(dg, sks)
    tr, want = ref.submit(pg.PG_OP_CN, 0, "and", u, v)
    ref.wait(tr)
    ref.close()
    for rep in range(2):
        held = [srv.submit(pg.PG_OP_CN, 0, "and", u, v) for _ in range(64)]  # 64 x 64 = the whole budget
        with pytest.raises(pg.PGError) as ei:
            srv.submit(pg.PG_OP_CN, 0, "and", u[:1], v[:1])
        assert ei.value.code == pg.PG_E_BUSY
        for t, out in held:
            srv.wait(t)
            assert out.tobytes() == want.tobytes()
    assert srv.stats()["completed"] == 128 and srv.stats()["rejected_busy"] == 2
    srv.close()


def test_malformed_requests_rejected_before_enqueue(env):
    g, ctx, dg, sks = env
    srv = pg.Server(dg, sks, max_pairs_per_request=100)
    ok = np.zeros(4, np.int32)
    bad = np.array([0, 1, g.n, 2], np.int32)
    cases = [(pg.PG_OP_CN, 0, "and", bad, ok), (pg.PG_OP_CN, 0, "kh", ok, ok), (pg.PG_OP_CN, 5, "and", ok, ok),
             (7, 0, "and", ok, ok), (pg.PG_OP_CN, 1, "kh", np.zeros(101, np.int32), np.zeros(101, np.int32)),
             (pg.PG_OP_CN, 0, "and", np.zeros(0, np.int32), np.zeros(0, np.int32))]
    for op, sk, est, u, v in cases:
        with pytest.raises(pg.PGError) as ei:
            srv.submit(op, sk, est, u, v)
        assert ei.value.code == pg.PG_E_INVALID
    assert srv.stats()["rejected_invalid"] == len(cases) and srv.stats()["submitted"] == 0
    srv.close()


def test_replay_open_and_closed_loop(env):
    g, ctx, dg, sks = env
    srv = pg.Server(dg, sks)
    reqs = [srv.make_request(op, sk, est, u, v) for op, sk, est, u, v in _requests(g, 60, seed=2)]
    lat, el = srv.replay(reqs, max_outstanding=8)
    assert np.all(lat > 0) and el > 0
    arrivals = np.cumsum(np.full(60, 1e-4))
    lat2, el2 = srv.replay(reqs, arrival_s=arrivals)
    assert np.all(lat2 > 0) and el2 >= arrivals[-1]
    assert srv.stats()["completed"] == 120
    # replayed results are the same as a direct call
    op, sk, est, u, v = _requests(g, 60, seed=2)[3]
    t, out = srv.submit(op, sk, est, u, v)
    srv.wait(t)
    assert out.tobytes() == reqs[3][1][2].tobytes()
    srv.close()


def test_alone_equals_mixed_with_concurrent_batches(env):
    """Every request of a mix replayed with three batch slots, small batches and
    many requests outstanding (so batches overlap on the device) returns
    bit for bit what it returns alone."""
    g, ctx, dg, sks = env
    reqs = _requests(g, 60, seed=5)
    srv = pg.Server(dg, sks, max_batches_in_flight=1)
    alone = []
    for op, sk, est, u, v in reqs:
        t, out = srv.submit(op, sk, est, u, v)
        srv.wait(t)
        alone.append(out.copy())
    srv.close()
    say("replaying the mix on three batch slots, batches of at most 4096 pairs")
    srv = pg.Server(dg, sks, max_batches_in_flight=3, max_pairs_per_request=4096, max_batch_pairs=4096)
    for rep in range(3):
        mix = [srv.make_request(op, sk, est, u, v) for op, sk, est, u, v in reqs]
        srv.replay(mix, max_outstanding=len(mix))
        for i, (a, (_, keep)) in enumerate(zip(alone, mix)):
            assert a.tobytes() == keep[2].tobytes(), (rep, i)
    st = srv.stats()
    assert st["completed"] == 3 * len(reqs)
    assert st["max_in_flight"] > 1, st  # batches did run concurrently
    srv.close()


def test_many_small_requests_in_one_batch(env):
    """Thousands of tiny requests queue behind long batches (three requests
    of 65,536 pairs in every 300), so batches hold more requests than travel as
    kernel arguments (their segment table is copied in front of the kernel)
    and up to the 1024 a batch holds; every answer equals the direct call's
    bit for bit."""
    g, ctx, dg, sks = env
    rng = np.random.default_rng(11)
    say("3000 requests of 1..4 pairs, three in every 300 of 65536 pairs, one batch slot")
    srv = pg.Server(dg, sks, max_batches_in_flight=1)
    kinds = [(0, "and"), (1, "kh"), (2, "1h")]
    spec = []
    for i in range(3000):
        long = i % 300 < 3  # three long 1-hash requests in a row
        L = 65536 if long else int(rng.integers(1, 5))
        u = rng.integers(0, g.n, L).astype(np.int32)
        v = rng.integers(0, g.n, L).astype(np.int32)
        sk, est = kinds[2] if long else kinds[i % 3]
        op = pg.PG_OP_CN if i % 2 == 0 else pg.PG_OP_JACCARD
        spec.append((op, sk, est, u, v))
    dev = torch.device("cuda", 0)
    for rep in range(5):
        mix = [srv.make_request(*s) for s in spec]
        srv.replay(mix, max_outstanding=len(mix))
        if srv.stats()["max_batch_requests"] > 128:
            break
    st = srv.stats()
    assert st["max_batch_requests"] > 128, st
    assert st["max_batch_requests"] <= 1024, st
    for (op, sk, est, u, v), (_, keep) in zip(spec, mix):
        tu, tv = torch.from_numpy(u).to(dev), torch.from_numpy(v).to(dev)
        direct = sks[sk].intersect(est, tu, tv)[0] if op == pg.PG_OP_CN else sks[sk].jaccard(est, tu, tv)
        torch.cuda.synchronize()
        assert direct.cpu().numpy().tobytes() == keep[2].tobytes()
    srv.close()
