"""The oracle's C half under AddressSanitizer and UndefinedBehaviorSanitizer:
a driver (tests/oracle_sanitize_main.c) runs every routine over a graph with
hubs, cliques, a star and isolated vertices; any invalid access or undefined
operation aborts it, and its counts must equal the regular oracle build's."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import pggen

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _graph():
    return pggen.disjoint_union(pggen.rmat(9, 8, seed=4), pggen.complete(9), pggen.star(40),
                                pggen.from_pairs(3, [], []), pggen.wheel(6))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_c_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitized"
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "oracle", "pg_oracle.c"), os.path.join(HERE, "oracle_sanitize_main.c"),
           "-lm", "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitizer" in (r.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    g = _graph()
    o = oracle.oriented(g)
    deg = np.diff(g.offsets).astype(np.int32)
    path = tmp_path / "graph.bin"
    with open(path, "wb") as f:
        f.write(np.int32(g.n).tobytes() + np.int64(g.nnz).tobytes())
        f.write(g.offsets.astype(np.int32).tobytes() + g.adj.astype(np.int32).tobytes())
        f.write(np.int64(o.nnz).tobytes() + o.offsets.astype(np.int32).tobytes() + o.adj.astype(np.int32).tobytes())
        f.write(deg.tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([str(exe), str(path)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    got = [int(x) for x in r.stdout.split()]

    eu, ev = oracle.upper_edges(g)
    bf = oracle.build_sketches(g, oracle.KIND_BF, 320, 2, 7)
    ca, co = bf.counts(eu, ev)
    kh = oracle.build_sketches(g, oracle.KIND_KH, 16, 1, 9)
    oh = oracle.build_sketches(g, oracle.KIND_1H, 16, 1, 11)
    su, kp, sl = oh.counts(eu, ev)
    pbf = oracle.build_sketches(o, oracle.KIND_BF, 128, 1, 5)
    want = [eu.shape[0], oracle.exact_tc_listing(g), int(oracle.exact_pairs(g, eu, ev).sum()), int(ca.sum()),
            int(co.sum()), int(bf.pc.sum()), int(kh.counts(eu, ev).sum()), int(su.sum()), int(kp.sum()),
            int(sl.sum()), oracle.four_cliques(g), oracle.four_cliques_bf(g, pbf)]
    ha, ho, sizes = oracle.four_cliques_filter_counts(g, pbf)
    c = np.arange(ha.shape[0], dtype=np.uint64)
    want += [int((ha * c).sum()), int((ho * c).sum()), sizes]
    assert got == want
