"""The benchmark's median confidence interval: distribution-free ranks from
the binomial(n, 1/2) distribution, checked against the textbook ranks."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_median_ci_ranks():
    b = _bench()
    # n = 30: x_(10) and x_(21), coverage 1 - 2 P(X <= 9) = 0.9572
    r = b.median_ci95([float(i) for i in range(30, 0, -1)])
    assert r["ci95_ms_per_step"] == [10.0, 21.0] and r["median_ms_per_step"] == 15.5
    assert abs(r["ci_coverage"] - 0.9572) < 1e-4
    # n = 100: x_(40) and x_(61)
    r = b.median_ci95([float(i) for i in range(1, 101)])
    assert r["ci95_ms_per_step"] == [40.0, 61.0]
    # n = 5: no pair of ranks reaches 95%, so the whole range, coverage 1 - 2/32
    r = b.median_ci95([3.0, 1.0, 2.0, 5.0, 4.0])
    assert r["ci95_ms_per_step"] == [1.0, 5.0] and r["median_ms_per_step"] == 3.0
    assert r["ci_coverage"] == 0.9375
