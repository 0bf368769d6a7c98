#!/usr/bin/env python3
"""Benchmark of the ProbGraph hot path on one MI355X.

Workload (the metric configuration): R-MAT scale 20, edge factor 16,
(a, b, c, d) = (0.57, 0.19, 0.19, 0.05), seed 1, symmetrized, deduplicated,
without self-loops; Bloom filters sized so all filter bits are 33% of the CSR
bytes, b = 1; triangle count by the AND estimator.

One step = the whole BF-sketch triangle-count job with the graph resident in
HBM: rebuild all n Bloom filters in place, estimate |N_u cap N_v| for all m
edges, reduce to TC^ (left in HBM; steps pipeline on the stream, one
synchronization closes the timed region). The synchronous variant, which
copies TC^ to the host every step, is reported beside it. value = m / step time (edge intersections
per second). Beside it: the HIP-event timing of the dominant kernel inside the
timed region (its roofline; the other phases are event-timed in an untimed
loop, since every bracketed launch costs device time), the exact GPU triangle count on the same
graph, the other rows of the path (b = 2, k-hash k = 32, clustering
coefficient, Jaccard) and the CPU oracle timed on this host.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "edge intersections/s (BF-sketch TC vs exact merge), R-MAT s20; query p50/p99"
UNIT = "edge intersections/s"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, public peak
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_bf_tc_rmat20.txt")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# sources the triangle-count kernel and its work plan are built from
TC_SOURCES = ("pg_estimate.hip", "pg_graph.hip", "pg_internal.h", "pg_device.h", "pg_pair.h")


def _src_hash(paths):
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def tc_source_hash():
    return _src_hash([os.path.join(ROOT, "paper_2208_11469_amd", "csrc", f) for f in TC_SOURCES])


def _read_traffic(B: int):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and not line.lstrip().startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != tc_source_hash() or int(kv.get("bf_bits", -1)) != B:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def timed(fn, reps, sync):
    """Median wall time (ms) of fn over reps, synchronizing around each call."""
    out = []
    for _ in range(reps):
        sync()
        t0 = time.perf_counter()
        fn()
        sync()
        out.append((time.perf_counter() - t0) * 1e3)
    return statistics.median(out)


def measure_batch(args, pg, pggen, np, torch, log):
    """Many small graphs: autotune, capture one run in a HIP graph, time replays."""
    t = time.perf_counter()
    graphs, bits = pggen.graph_batch(count=args.batch_graphs, seed0=args.seed)
    n_total = sum(g.n for g in graphs)
    arcs = sum(g.nnz for g in graphs)
    log(f"batch: {len(graphs)} graphs, {n_total} vertices, {arcs} arcs ({time.perf_counter() - t:.1f}s)")
    ctx = pg.Context(0)
    bt = pg.Batch(ctx, graphs, bits, b=1, seed=args.seed)
    tune_ms = bt.autotune("and")
    tile, bpc = bt.params()
    s = torch.cuda.Stream()
    bt.capture("and", stream=s)
    for _ in range(3):
        bt.replay(stream=s)
    torch.cuda.synchronize()
    times = []
    for _ in range(20):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        bt.replay(stream=s)
        e1.record(s)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = statistics.median(times)
    tc, _ = bt.results(stream=s)
    # bytes the method moves per run: build reads offsets and arcs and writes rows; the estimate reads
    # offsets, arcs, its own row and one neighbour row per arc
    row_bytes = sum(g.n * (B // 8) for g, B in zip(graphs, bits))
    nbr_rows = sum(g.nnz * (B // 8) for g, B in zip(graphs, bits))
    alg = 2 * (8 * n_total + 4 * arcs) + 2 * row_bytes + 4 * n_total + nbr_rows + 8 * n_total * 3
    bt.close()
    ctx.close()
    log(f"batch replay {ms:.3f} ms ({arcs / (ms * 1e-3):.3e} arc intersections/s), tile {tile} blocks/CU {bpc}")
    return {"workload": f"{len(graphs)} graphs, n log-uniform in [2^8, 2^16], half G(n,p) (mean degree 8..64), "
                        "half R-MAT ef16; BF 128..1024 bits b=1; TC + CC per graph, AND estimator",
            "graphs": len(graphs), "vertices": n_total, "arcs": arcs, "replay_ms": round(ms, 4),
            "arc_intersections_per_s": arcs / (ms * 1e-3), "algorithmic_gbs": alg / (ms * 1e-3) / 1e9,
            "autotuned": {"tile_vertices": tile, "blocks_per_cu": bpc, "best_ms": round(tune_ms, 4)},
            "tc_sum": float(np.sum(tc))}


def measure_serving(args, pg, pggen, np, log):
    """Query serving on a resident R-MAT graph: closed-loop saturation, then
    open-loop Poisson arrivals at 50/80/95% of it; latency from arrival to
    result on the host."""
    t = time.perf_counter()
    g = pggen.rmat(args.serving_scale, 16, seed=args.seed)
    ctx = pg.Context(0)
    dg = pg.Graph(ctx, g.offsets, g.adj)
    sks = [dg.build_sketches("bf", 512, 1, seed=args.seed), dg.build_sketches("kh", 32, seed=args.seed)]
    log(f"serving: R-MAT s{args.serving_scale} n={g.n} nnz={g.nnz} resident with BF-512 and k-hash-32 "
        f"({time.perf_counter() - t:.1f}s)")
    trace = pggen.query_trace(g.n, args.serving_requests, rate_hz=1.0, seed=args.seed)
    srv = pg.Server(dg, sks, max_batches_in_flight=3)
    reqs = []
    for r in trace:
        op = pg.PG_OP_CN if r.op == "cn" else pg.PG_OP_JACCARD
        sk, est = (0, "and") if r.kind == "bf" else (1, "kh")
        reqs.append(srv.make_request(op, sk, est, r.u, r.v))
    pairs = sum(int(r.u.shape[0]) for r in trace)
    mean_pairs = pairs / len(trace)
    # algorithmic bytes of the trace (two sketch rows, two IDs and the answer
    # per pair; two degrees more for Jaccard and MinHash) and bus bytes (the
    # pair IDs read from and the answer written to pinned host memory)
    row = {"bf": 512 // 8, "mh": 4 * 32}
    alg = sum(int(r.u.shape[0]) * (2 * row[r.kind] + 8 + (8 if r.op == "cn" else 4)
                                   + (8 if (r.op == "jaccard" or r.kind == "mh") else 0)) for r in trace)
    bus = sum(int(r.u.shape[0]) * (8 + (8 if r.op == "cn" else 4)) for r in trace)
    srv.replay(reqs[: min(200, len(reqs))], max_outstanding=32)  # warm-up
    reps = 5  # the closed-loop saturation replays the trace several times
    el = 0.0
    for _ in range(reps):
        lat, e = srv.replay(reqs, max_outstanding=args.serving_outstanding)
        el += e
    sat_pairs = reps * pairs / el
    sat_rate = reps * len(reqs) / el
    sat_hbm = reps * alg / el / 1e9
    sat_bus = reps * bus / el / 1e9
    log(f"serving saturation ({args.serving_outstanding} outstanding): {sat_pairs:.3e} pairs/s, {sat_rate:.0f} requests/s, "
        f"{sat_hbm:.1f} GB/s algorithmic, "
        f"p50 {np.percentile(lat, 50):.3f} ms")
    unit_gaps = np.diff(np.concatenate([[0.0], [r.arrival_s for r in trace]]))  # Poisson gaps at 1 request/s
    loads = []
    for frac in (0.5, 0.8, 0.95):
        rate = frac * sat_rate
        arrivals = np.cumsum(unit_gaps / rate)
        lat, el = srv.replay(reqs, arrival_s=arrivals)
        loads.append({"load": frac, "rate_requests_per_s": rate, "p50_ms": float(np.percentile(lat, 50)),
                      "p99_ms": float(np.percentile(lat, 99)), "pairs_per_s": pairs / el})
        log(f"serving at {frac:.0%}: p50 {loads[-1]['p50_ms']:.3f} ms p99 {loads[-1]['p99_ms']:.3f} ms")
    st = srv.stats()
    srv.close()
    for sk in sks:
        sk.close()
    dg.close()
    ctx.close()
    return {"workload": f"R-MAT s{args.serving_scale} ef16 resident, BF 512 bits b=1 + k-hash k=32; "
                        f"{len(reqs)} Poisson requests, 1..65536 pairs (log-uniform), CN/Jaccard x BF/MH",
            "mean_pairs_per_request": mean_pairs, "saturation_pairs_per_s": sat_pairs,
            "saturation_requests_per_s": sat_rate, "saturation_outstanding": args.serving_outstanding,
            "saturation_algorithmic_gbs": round(sat_hbm, 2), "saturation_frac_hbm": round(sat_hbm / HBM_PEAK_GBS, 5),
            "saturation_bus_gbs": round(sat_bus, 2),
            "bytes_rule": "per pair 2 rows (BF-512: 64 B, k-hash-32: 128 B) + 8 (IDs) + answer (8 CN, 4 Jaccard) "
                          "+ 8 (degrees, Jaccard or MinHash); bus: 8 (IDs) + answer",
            "loads": loads, "batches": st["batches"], "max_batches_in_flight": st["max_in_flight"],
            "requests": st["completed"]}


def kernel_ms(pg, ctx, site, fn, reps, sync):
    """Average device time of launch site `site` over reps calls of fn (HIP events)."""
    sync()
    pg.pg_profile_reset(ctx.h)
    pg.pg_profile_select(ctx.h, site)
    pg.pg_profile_enable(ctx.h, True)
    for _ in range(reps):
        fn()
    sync()
    pg.pg_profile_enable(ctx.h, False)
    launches, total = pg.pg_profile_read(ctx.h).get(site, (0, 0.0))
    pg.pg_profile_select(ctx.h, None)
    pg.pg_profile_reset(ctx.h)
    return total / launches if launches else float("nan")


def measure_scale24(args, pg, pggen, torch, ctx, sync, log):
    """R-MAT scale 24, edge factor 32 (about 1e9 arcs): 1024-bit Bloom filters and
    1-hash k = 64, triangle count and clustering coefficient, exact GPU merge
    baseline. The exact clustering coefficient (tens of seconds) and the bitmap
    triangle count (minutes) run only with --scale24-slow."""
    t = time.perf_counter()
    g = pggen.rmat(24, 32, seed=args.seed)
    log(f"scale24: generated n={g.n} nnz={g.nnz} ({time.perf_counter() - t:.1f}s)")
    dg = pg.Graph(ctx, g.offsets, g.adj)
    m = dg.m
    log(f"scale24: graph resident, m={m}")
    out = {"workload": f"R-MAT s24 ef32 (0.57,0.19,0.19,0.05) seed {args.seed}; n={g.n} m={m} nnz={g.nnz}"}
    exact_tc = dg.exact_tc()  # builds the degree orientation once
    exact_ms = timed(lambda: dg.exact_tc(), 3, sync)
    out["exact"] = {"tc": exact_tc, "tc_ms": round(exact_ms, 3), "intersections_per_s": m / (exact_ms * 1e-3)}
    log(f"scale24 exact TC {exact_tc} in {exact_ms:.1f} ms")
    if args.scale24_slow:
        t0 = time.perf_counter()
        dg.exact_cc()
        sync()
        out["exact"]["cc_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
        log(f"scale24 exact CC in {out['exact']['cc_ms']:.1f} ms")
        t0 = time.perf_counter()
        assert dg.exact_tc(algo=pg.PG_EXACT_BITMAP) == exact_tc
        out["exact"]["tc_bitmap_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
        log(f"scale24 exact TC by bitmap in {out['exact']['tc_bitmap_ms']:.1f} ms")
    for name, kind, size, est, site, row_bytes in (("bf1024", "bf", 1024, "and", "bf_tc", 128),
                                                   ("onehash64", "1h", 64, "1h", "oh_tc", 256)):
        sk = dg.build_sketches(kind, size, 1, seed=args.seed)
        tc = sk.tc(est)  # first call builds the triangle-count plan
        b_ms = timed(lambda: sk.rebuild(), 5, sync)
        t_ms = timed(lambda: sk.tc(est), 5, sync)
        c_ms = timed(lambda: sk.cc(est), 3, sync)
        k_ms = kernel_ms(pg, ctx, site, lambda: sk.tc(est), 3, sync)
        # per edge two rows and two IDs (plus two degrees for the MinHash estimate)
        per_edge = 2 * row_bytes + 8 + (8 if kind == "1h" else 0)
        gbs = m * per_edge / (k_ms * 1e-3) / 1e9
        out[name] = {"build_ms": round(b_ms, 3), "tc_ms": round(t_ms, 3), "cc_ms": round(c_ms, 3),
                     "tc_kernel_ms": round(k_ms, 3),
                     "tc_kernel_algorithmic": {"bytes_per_edge": per_edge, "gbs": round(gbs, 1),
                                               "frac_of_8tbs": round(gbs / HBM_PEAK_GBS, 4)},
                     "step_intersections_per_s": m / ((b_ms + t_ms) * 1e-3),
                     "estimate_intersections_per_s": m / (t_ms * 1e-3), "tc": tc,
                     "rel_err": abs(tc - exact_tc) / exact_tc, "speedup_vs_exact": exact_ms / (b_ms + t_ms)}
        log(f"scale24 {name}: build {b_ms:.2f} ms, TC {t_ms:.2f} ms (kernel {k_ms:.2f}), CC {c_ms:.2f} ms, "
            f"rel err {abs(tc - exact_tc) / exact_tc:.3e}")
        sk.close()
    dg.close()
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def measure_cpu(args, g, B, m, tc_bf, exact_tc, exact_gpu_ms, log):
    """The oracle on this host's cores: BF build + AND estimate of every edge +
    TC sum (all cores, median of 3; and on one core), and the exact merge
    triangle count of the node iterator (all cores, once)."""
    import oracle
    all_threads = oracle.threads()
    times, tc_cpu = [], None
    for _ in range(3):
        t = time.perf_counter()
        ref = oracle.build_sketches(g, oracle.KIND_BF, B, args.b, seed=args.seed)
        tc_cpu = oracle.tc(ref, "and")
        times.append(time.perf_counter() - t)
        del ref
    cpu_s = statistics.median(times)
    oracle.set_threads(1)
    t = time.perf_counter()
    ref = oracle.build_sketches(g, oracle.KIND_BF, B, args.b, seed=args.seed)
    tc_one = oracle.tc(ref, "and")
    one_s = time.perf_counter() - t
    del ref
    oracle.set_threads(all_threads)
    t = time.perf_counter()
    ex = oracle.exact_tc_listing(g)
    ex_s = time.perf_counter() - t
    assert ex == exact_tc, (ex, exact_tc)
    log(f"cpu oracle ({cpu_model()}): BF TC {cpu_s:.3f} s on {all_threads} threads, {one_s:.3f} s on 1; "
        f"exact merge TC {ex_s:.3f} s")
    return {"value": m / cpu_s, "unit": UNIT, "cores": all_threads, "kind": "oracle",
            "sample": "full workload: oracle BF build (b=1, same B and seed) + AND counts and FP64 estimates "
                      "for all m edges + TC sum; median of 3",
            "seconds": round(cpu_s, 4), "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "tc_matches_gpu_rel": abs(tc_cpu - tc_bf) / abs(tc_cpu),
            "single_core": {"seconds": round(one_s, 4), "value": m / one_s, "unit": UNIT, "cores": 1,
                            "tc_equal": tc_one == tc_cpu},
            "exact_merge_tc": {"seconds": round(ex_s, 4), "edge_intersections_per_s": m / ex_s,
                               "cores": all_threads, "tc": ex,
                               "algorithm": "degree-ordered node iterator, sorted merge per oriented edge",
                               "gpu_exact_speedup": ex_s / (exact_gpu_ms * 1e-3)}}


def measure_c0(args, pg, pggen, torch, ctx, sync, log):
    """The small parity configuration: G(n, p), n = 4096, mean degree 16, seed 1;
    256-bit Bloom filters, b = 1; AND and limit estimates of the triangle count
    against the exact count (launch-latency bound, not a roofline case)."""
    g = pggen.er(4096, 16, seed=args.seed)
    dg = pg.Graph(ctx, g.offsets, g.adj)
    sk = dg.build_sketches("bf", 256, 1, seed=args.seed)
    exact = dg.exact_tc()
    out = {"workload": f"G(n,p) n=4096 mean degree 16 seed {args.seed}; BF 256 bits b=1", "n": g.n, "m": dg.m,
           "tc_exact": exact, "exact_ms": round(timed(lambda: dg.exact_tc(), 10, sync), 4)}
    for est in ("and", "l"):
        tc = sk.tc(est)
        ms = timed(lambda: (sk.rebuild(), sk.tc(est)), 10, sync)
        out[f"tc_{est}"] = {"tc": tc, "rel_err": abs(tc - exact) / exact if exact else None, "ms_per_call": round(ms, 4)}
    sk.close()
    dg.close()
    log(f"C0: exact {exact}, AND {out['tc_and']['tc']:.1f}, limit {out['tc_l']['tc']:.1f}")
    return out


def median_ci95(x):
    """Median of the samples and a distribution-free 95% confidence interval
    for it: the order statistics x_(k), x_(n-k+1) with k the largest rank
    such that P(Bin(n, 1/2) <= k - 1) <= 0.025 (coverage >= 95%)."""
    x = sorted(x)
    n = len(x)
    cdf, k = 0.0, 0
    while cdf + math.comb(n, k) / 2.0**n <= 0.025:
        cdf += math.comb(n, k) / 2.0**n
        k += 1
    if k >= 1:
        lo, hi, coverage = x[k - 1], x[n - k], 1.0 - 2.0 * cdf
    else:  # too few samples: the whole range, whose coverage falls short of 95%
        lo, hi, coverage = x[0], x[-1], 1.0 - 2.0 / 2.0**n
    med = x[n // 2] if n % 2 else 0.5 * (x[n // 2 - 1] + x[n // 2])
    return {"median_ms_per_step": round(med, 5), "ci95_ms_per_step": [round(lo, 5), round(hi, 5)],
            "ci_coverage": round(coverage, 4), "min_ms_per_step": round(x[0], 5),
            "max_ms_per_step": round(x[-1], 5)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--edge-factor", type=int, default=16)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--budget", type=float, default=0.33)
    ap.add_argument("--b", type=int, default=1)
    ap.add_argument("--skip-cpu", action="store_true", help="leave out the CPU oracle baseline")
    ap.add_argument("--skip-rows", action="store_true", help="leave out the extra rows")
    ap.add_argument("--rows", default=None, help="comma-separated names of the extra rows to run (default: all)")
    ap.add_argument("--skip-serving", action="store_true", help="leave out the serving measurement")
    ap.add_argument("--serving-scale", type=int, default=22)
    ap.add_argument("--serving-requests", type=int, default=10000)
    ap.add_argument("--skip-batch", action="store_true", help="leave out the batched-graphs measurement")
    ap.add_argument("--serving-outstanding", type=int, default=512,
                    help="requests kept outstanding in the closed-loop saturation replay (the measured "
                         "throughput levels off from about 256 on: 3.1 / 3.2 / 3.3e9 pairs/s at 256 / 384 / 512)")
    ap.add_argument("--batch-graphs", type=int, default=512)
    ap.add_argument("--skip-scale24", action="store_true",
                    help="leave out the R-MAT s24 ef32 configuration (BF-1024, 1-hash-64, exact merge)")
    ap.add_argument("--scale24-slow", action="store_true",
                    help="in the s24 configuration also time the exact CC and the bitmap exact TC (minutes)")
    ap.add_argument("--skip-c0", action="store_true", help="leave out the small G(n,p) configuration")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the ProbGraph path here is built and timed on a single "
              "MI355X (the multi-GPU plan is a design note, not a measured configuration). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2208_11469_amd as pg
    import pggen

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    sync = torch.cuda.synchronize

    t = time.perf_counter()
    g = pggen.rmat(args.scale, args.edge_factor, seed=args.seed)
    log(f"generated R-MAT s{args.scale} ef{args.edge_factor}: n={g.n} nnz={g.nnz} ({time.perf_counter() - t:.1f}s)")
    ctx = pg.Context(0)
    dg = pg.Graph(ctx, g.offsets, g.adj)
    n, m, nnz = dg.n, dg.m, dg.nnz
    B = dg.bits_for_budget(args.budget)
    S = B // 8
    sk = dg.build_sketches("bf", B, args.b, seed=args.seed)
    log(f"graph resident: m={m} max_degree={dg.max_degree}; BF B={B} bits b={args.b}")

    d_tc = torch.zeros(1, dtype=torch.float64, device=dev)

    def step():
        # the whole job on the stream; steps pipeline, the result stays in HBM
        sk.rebuild()
        sk.tc_async("and", d_tc)

    for _ in range(args.warmup):
        step()
    sync()
    # inside the timed region only the dominant kernel is bracketed by HIP
    # events (each recorded launch costs device time between launches); the
    # other phases are timed in an untimed loop below
    pg.pg_profile_reset(ctx.h)
    pg.pg_profile_select(ctx.h, "bf_tc")
    pg.pg_profile_enable(ctx.h, True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    sync()
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    sync()
    wall_ms = (time.perf_counter() - t0) * 1e3
    pg.pg_profile_enable(ctx.h, False)
    prof = pg.pg_profile_read(ctx.h)
    pg.pg_profile_select(ctx.h, None)
    ms_per_step = wall_ms / args.steps
    # every phase of the step, in an untimed loop of its own
    pg.pg_profile_reset(ctx.h)
    pg.pg_profile_enable(ctx.h, True)
    for _ in range(min(args.steps, 20)):
        step()
    sync()
    pg.pg_profile_enable(ctx.h, False)
    prof_phases = pg.pg_profile_read(ctx.h)
    pg.pg_profile_reset(ctx.h)
    # repetitions for the median and its 95% non-parametric confidence
    # interval (the paper's reporting), each rep of 10 steps bracketed by HIP
    # events on the launch stream; `value` stays the timed region above
    rep_ms = []
    for _ in range(30):
        r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        r0.record()
        for _ in range(10):
            step()
        r1.record()
        r1.synchronize()
        rep_ms.append(r0.elapsed_time(r1) / 10)
    step_stats = {"reps": len(rep_ms), "steps_per_rep": 10, **median_ci95(rep_ms),
                  "timer": "HIP events on the launch stream"}
    value = m / (ms_per_step * 1e-3)
    tc_bf = float(d_tc.item())
    tc_sync = sk.tc("and")
    assert tc_sync == tc_bf, (tc_sync, tc_bf)
    sync_ms = timed(lambda: (sk.rebuild(), sk.tc("and")), 20, sync)
    log(f"timed {args.steps} steps: {ms_per_step:.4f} ms/step -> {value:.4e} {UNIT}; kernels {prof}")

    def avg(name, source=None):
        launches, total = (prof if source is None else source).get(name, (0, 0.0))
        return total / launches if launches else float("nan")

    # roofline of the dominant kernel, the vertex-centric edge-estimate sum.
    # Algorithmic bytes by the per-intersection rule: two sketch rows and the
    # two endpoint IDs per edge, 2S + 8. The kernel keeps the owner's row in
    # registers across its upper edges, so it requests fewer bytes than that:
    # per upper edge the neighbour ID and its row, per vertex with upper edges
    # its own row, ustart and two offsets (the reuse-aware figure); and of those
    # requests the caches serve part (the counter-measured HBM bytes).
    deg = np.diff(g.offsets).astype(np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), deg)
    n_active = int(np.count_nonzero(np.bincount(src[g.adj > src], minlength=n)))
    del src
    alg_bytes = m * (2 * S + 8)
    reuse_bytes = m * (S + 4) + n_active * (S + 12)
    k_ms = avg("bf_tc")
    achieved = alg_bytes / (k_ms * 1e-3) / 1e9
    traffic = _read_traffic(B)
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_bf_tc_slab (AND count + estimate over every upper edge, XCD-sliced vertex plan)",
                "kernel_ms": round(k_ms, 5), "algorithmic_bytes": alg_bytes, "bytes_rule": "m*(2S+8), S = B/8",
                "frac_note": "above 1: the rows are re-read from the caches (the 44.7 MB filter array fits the "
                             "256 MB Infinity Cache), so the per-intersection rule is an effective bandwidth",
                "reuse_aware": {"bytes": reuse_bytes, "bytes_rule": "m*(S+4) + n_active*(S+12)",
                                "gbs": round(reuse_bytes / (k_ms * 1e-3) / 1e9, 2),
                                "frac": round(reuse_bytes / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
                "hbm_measured": None if traffic is None else {
                    "bytes": traffic, "gbs": round(traffic / (k_ms * 1e-3) / 1e9, 2),
                    "frac": round(traffic / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "source": os.path.relpath(TRAFFIC_FILE, ROOT)}}
    build_ms = avg("bf_build", prof_phases)
    # build: offsets (two per vertex), every arc's ID, the row and popcount, the plan lists
    build_bytes = 8 * n + 4 * nnz + n * S + 4 * n + 4 * n
    phases = {name: {"launches": c, "avg_ms": round(tot / c, 5)} for name, (c, tot) in prof_phases.items() if c}

    # exact GPU baseline on the same graph (orientation built once, outside the timing)
    exact_tc = dg.exact_tc()
    exact_ms = timed(lambda: dg.exact_tc(), 5, sync)
    rel_err = abs(tc_bf - exact_tc) / exact_tc if exact_tc else float("nan")
    log(f"exact TC {exact_tc} in {exact_ms:.3f} ms; BF-AND TC^ {tc_bf:.1f} (rel err {rel_err:.3f})")

    # reference copy bandwidth
    nb = 1 << 30
    src = torch.empty(nb, dtype=torch.uint8, device=dev)
    dst = torch.empty(nb, dtype=torch.uint8, device=dev)
    pg.pg_copy(ctx.h, dst, src, nb)
    copy_ms = timed(lambda: pg.pg_copy(ctx.h, dst, src, nb), 10, sync)
    copy_gbs = 2 * nb / (copy_ms * 1e-3) / 1e9
    del src, dst

    rows = {}
    sel = set(args.rows.split(",")) if args.rows else None

    def want(*names):
        return not args.skip_rows and (sel is None or any(k in sel for k in names))

    reps = 10
    if want("bf_b2_tc"):
        # b = 2 at the same budget
        sk2 = dg.build_sketches("bf", B, 2, seed=args.seed)
        ms = timed(lambda: (sk2.rebuild(), sk2.tc("and")), reps, sync)
        tc2 = sk2.tc("and")
        rows["bf_b2_tc"] = {"ms": round(ms, 4), "intersections_per_s": m / (ms * 1e-3), "tc": tc2,
                            "rel_err": abs(tc2 - exact_tc) / exact_tc}
        sk2.close()
    if want("khash32_tc", "khash32_jaccard_edges", "khash32_cc"):
        # k-hash, k = 32
        skk = dg.build_sketches("kh", 32, seed=args.seed)
        ms_b = timed(lambda: skk.rebuild(), reps, sync)
        ms_t = timed(lambda: skk.tc("kh"), reps, sync)
        tck = skk.tc("kh")
        rows["khash32_tc"] = {"build_ms": round(ms_b, 4), "tc_ms": round(ms_t, 4),
                              "intersections_per_s": m / ((ms_b + ms_t) * 1e-3), "tc": tck,
                              "rel_err": abs(tck - exact_tc) / exact_tc}
        ms = timed(lambda: skk.jaccard("kh"), reps, sync)
        rows["khash32_jaccard_edges"] = {"ms": round(ms, 4), "intersections_per_s": m / (ms * 1e-3)}
        ms = timed(lambda: skk.cc("kh"), reps, sync)
        rows["khash32_cc"] = {"ms": round(ms, 4), "arc_intersections_per_s": nnz / (ms * 1e-3)}
        skk.close()
    if want("bf_oriented_tc"):
        # sketches of the degree-oriented sets N+_v (node iterator form of the
        # triangle count): same sizes, smaller sets
        sko = dg.build_sketches("bf", B, 1, seed=args.seed, oriented=True)
        ms = timed(lambda: (sko.rebuild(), sko.tc("and")), reps, sync)
        tco = sko.tc("and")
        rows["bf_oriented_tc"] = {"ms": round(ms, 4), "intersections_per_s": m / (ms * 1e-3), "tc": tco,
                                  "rel_err": abs(tco - exact_tc) / exact_tc}
        sko.close()
    if want("khash32_oriented_tc"):
        sko = dg.build_sketches("kh", 32, seed=args.seed, oriented=True)
        ms_b = timed(lambda: sko.rebuild(), reps, sync)
        ms_t = timed(lambda: sko.tc("kh"), reps, sync)
        tco = sko.tc("kh")
        rows["khash32_oriented_tc"] = {"build_ms": round(ms_b, 4), "tc_ms": round(ms_t, 4),
                                       "intersections_per_s": m / ((ms_b + ms_t) * 1e-3), "tc": tco,
                                       "rel_err": abs(tco - exact_tc) / exact_tc}
        sko.close()
    # KMV estimators on 1-hash rows, k = 32, full and oriented sets
    for key, oriented in (("kmv32_tc", False), ("kmv32_oriented_tc", True)):
        if want(key):
            skm = dg.build_sketches("1h", 32, seed=args.seed, oriented=oriented)
            ms_b = timed(lambda: skm.rebuild(), reps, sync)
            ms_t = timed(lambda: skm.tc("kmv"), reps, sync)
            tcm = skm.tc("kmv")
            rows[key] = {"build_ms": round(ms_b, 4), "tc_ms": round(ms_t, 4),
                         "intersections_per_s": m / ((ms_b + ms_t) * 1e-3), "tc": tcm,
                         "rel_err": abs(tcm - exact_tc) / exact_tc,
                         "tc_1hash_union": skm.tc("1h"), "tc_kmv_sketch_sizes": skm.tc("kmv_est")}
            skm.close()
    if want("four_cliques"):
        # 4-cliques: exact, and with membership queries on the filters of N+_v
        sko = dg.build_sketches("bf", B, 1, seed=args.seed, oriented=True)
        ck_bf = sko.four_cliques()
        ms_bf = timed(lambda: sko.four_cliques(), 5, sync)
        ck_and = sko.four_cliques_estimate("and")
        ms_and = timed(lambda: sko.four_cliques_estimate("and"), 5, sync)
        ck_l = sko.four_cliques_estimate("l")
        ck_ex = dg.exact_four_cliques()
        ms_ex = timed(lambda: dg.exact_four_cliques(), 3, sync)
        rows["four_cliques"] = {"bf_ms": round(ms_bf, 4), "exact_ms": round(ms_ex, 4), "bf": ck_bf, "exact": ck_ex,
                                "rel_err": (ck_bf - ck_ex) / max(ck_ex, 1), "speedup_bf_vs_exact": ms_ex / ms_bf,
                                "bf_and_ms": round(ms_and, 4), "bf_and": ck_and, "bf_limit": ck_l,
                                "rel_err_and": (ck_and - ck_ex) / max(ck_ex, 1),
                                "rel_err_limit": (ck_l - ck_ex) / max(ck_ex, 1),
                                "speedup_bf_and_vs_exact": ms_ex / ms_and}
        sko.close()
    if want("bf_cc", "bf_jaccard_edges"):
        # clustering coefficient and Jaccard (BF AND, b = 1)
        ms = timed(lambda: sk.cc("and"), reps, sync)
        rows["bf_cc"] = {"ms": round(ms, 4), "arc_intersections_per_s": nnz / (ms * 1e-3)}
        ms = timed(lambda: sk.jaccard("and"), reps, sync)
        rows["bf_jaccard_edges"] = {"ms": round(ms, 4), "intersections_per_s": m / (ms * 1e-3)}
    if want("exact_edges", "exact_cc"):
        # exact per-edge intersections (all m edges) and exact CC
        ms = timed(lambda: dg.exact_intersect(), 3, sync)
        rows["exact_edges"] = {"ms": round(ms, 4), "intersections_per_s": m / (ms * 1e-3)}
        ms = timed(lambda: dg.exact_cc(), 3, sync)
        rows["exact_cc"] = {"ms": round(ms, 4)}
    if want("accuracy_bf_and"):
        # accuracy of the BF AND estimates on every edge and vertex: per-edge
        # relative error where I > 0, mean absolute error where I = 0, CC mean
        # absolute error, Jaccard absolute error quantiles
        qs = (0.05, 0.25, 0.5, 0.75, 0.95)

        def quantiles(t):
            t = torch.sort(t.flatten())[0]
            return [round(float(t[int(q * (t.numel() - 1))]), 5) for q in qs] if t.numel() else []

        i_ex = dg.exact_intersect().double()
        i_bf = sk.intersect("and", want_raw=False)[0].double()
        pos = i_ex > 0
        rows["accuracy_bf_and"] = {
            "quantiles": list(qs),
            "edges_I_pos": int(pos.sum()), "edges_I_zero": int((~pos).sum()),
            "intersection_rel_err_I_pos": quantiles((i_bf[pos] - i_ex[pos]).abs() / i_ex[pos]),
            "intersection_mae_I_zero": round(float(i_bf[~pos].abs().mean()), 5) if bool((~pos).any()) else None,
            "cc_mae": round(float((sk.cc("and").double() - dg.exact_cc().double()).abs().mean()), 6),
            "jaccard_abs_err": quantiles((sk.jaccard("and").double() - dg.exact_jaccard().double()).abs())}
        del i_ex, i_bf, pos
    if want("exact_edges_bitmap", "exact_tc_bitmap"):
        # the bitmap variant of the exact baseline (all upper edges; triangle count)
        ms = timed(lambda: dg.exact_intersect(algo=pg.PG_EXACT_BITMAP), 3, sync)
        rows["exact_edges_bitmap"] = {"ms": round(ms, 4), "intersections_per_s": m / (ms * 1e-3)}
        assert dg.exact_tc(algo=pg.PG_EXACT_BITMAP) == exact_tc
        ms = timed(lambda: dg.exact_tc(algo=pg.PG_EXACT_BITMAP), 3, sync)
        rows["exact_tc_bitmap"] = {"ms": round(ms, 4), "intersections_per_s": m / (ms * 1e-3)}
    for mname, tau in (("cn", 8.5), ("jaccard", 0.05), ("overlap", 0.5)):
        if not want(f"jarvis_patrick_{mname}"):
            continue
        # Jarvis-Patrick clustering over all m edges (similarity > tau) and its
        # clusters, from the filters and exactly (merge); accuracy as the
        # relative error of the counts
        keep_b, kept_b = sk.jarvis_patrick("and", mname, tau)
        ms_b = timed(lambda: sk.jarvis_patrick("and", mname, tau), reps, sync)
        ncl_b = dg.clusters(keep_b)[1]
        ms_c = timed(lambda: dg.clusters(keep_b), reps, sync)
        keep_x, kept_x = dg.exact_jarvis_patrick(mname, tau)
        ms_x = timed(lambda: dg.exact_jarvis_patrick(mname, tau), 3, sync)
        ncl_x = dg.clusters(keep_x)[1]
        rows[f"jarvis_patrick_{mname}"] = {
            "tau": tau, "bf_ms": round(ms_b, 4), "bf_edges_per_s": m / (ms_b * 1e-3),
            "clusters_ms": round(ms_c, 4), "exact_ms": round(ms_x, 4),
            "speedup_bf_vs_exact": (ms_x + ms_c) / (ms_b + ms_c),
            "kept_bf": kept_b, "kept_exact": kept_x, "clusters_bf": ncl_b, "clusters_exact": ncl_x,
            "cluster_count_rel_err": abs(ncl_b - ncl_x) / max(ncl_x, 1)}
        del keep_b, keep_x

    cpu = None
    if not args.skip_cpu:
        cpu = measure_cpu(args, g, B, m, tc_bf, exact_tc, exact_ms, log)
    batch = None
    if not args.skip_batch:
        batch = measure_batch(args, pg, pggen, np, torch, log)

    serving = None
    if not args.skip_serving:
        serving = measure_serving(args, pg, pggen, np, log)

    c0 = None if args.skip_c0 else measure_c0(args, pg, pggen, torch, ctx, sync, log)

    scale24 = None if args.skip_scale24 else measure_scale24(args, pg, pggen, torch, ctx, sync, log)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"R-MAT s{args.scale} ef{args.edge_factor} (0.57,0.19,0.19,0.05) seed {args.seed}; "
                               f"BF-sketch TC, AND estimator, {int(args.budget * 100)}% storage budget",
                   "n": n, "m": m, "nnz": nnz, "bf_bits": B, "b": args.b,
                   "step": "rebuild n filters + estimate m edges + TC reduce"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "tc_estimate": tc_bf,
        "tc_exact": exact_tc,
        "tc_rel_err": rel_err,
        "exact_gpu": {"tc_ms": round(exact_ms, 4), "intersections_per_s": m / (exact_ms * 1e-3),
                      "speedup_bf_vs_exact": exact_ms / ms_per_step},
        "bf_build": {"avg_ms": round(build_ms, 5), "bytes": build_bytes,
                     "gbs": round(build_bytes / (build_ms * 1e-3) / 1e9, 2)},
        "estimate_only_intersections_per_s": m / ((avg("bf_tc") + avg("sum_chunks", prof_phases)) * 1e-3),
        "ms_per_step_synchronous": round(sync_ms, 4),
        "copy_kernel_gbs": round(copy_gbs, 1),
        "phases": phases,
        "step_stats": step_stats,
        "rows": rows,
        "serving": serving,
        "batch": batch,
        "c0": c0,
        "scale24": scale24,
    }
    print(json.dumps(out), flush=True)
    sk.close()
    dg.close()


if __name__ == "__main__":
    main()
