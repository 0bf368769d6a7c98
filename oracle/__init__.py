"""ProbGraph reference oracle (FP64 / exact integers, CPU).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. The GPU library
never calls it; it shares no code, header, table or constant generator with it.

Integer quantities (exact intersections, sketches, bit and match counts) come
from ``pg_oracle.c``; the estimator formulas are written out below in FP64
numpy, each next to the passage of the paper it follows.

Functions whose result has no external pin are marked "parity unpinned".
Every other function is pinned by ``tests/test_oracle_*.py`` against closed
forms, brute force, published test vectors or the statistics the paper states.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pg_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libpgoracle.so")
_lib = None

BOTTOM = 0xFFFFFFFF
KIND_BF, KIND_KH, KIND_1H = 1, 2, 3

BF_ESTIMATORS = ("and", "l", "or", "pap")
MH_ESTIMATORS = {"kh": KIND_KH, "1h": KIND_1H, "1h_lit": KIND_1H, "kmv": KIND_1H, "kmv_est": KIND_1H}


def build() -> str:
    """Compile the oracle's C half (gcc, OpenMP)."""
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC, "-lm", "-o", tmp])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    i32p = ctypes.POINTER(ctypes.c_int32)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    u64, i32, i64, u32 = ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    sig = {
        "or_threads": (ctypes.c_int, []),
        "or_set_threads": (None, [ctypes.c_int]),
        "or_splitmix64": (u64, [u64, u64]),
        "or_hash_consts": (None, [ctypes.c_int, u64, ctypes.c_int, u64p, u64p]),
        "or_bf_index": (u32, [u64, u64, u32, u32]),
        "or_mh_key": (u64, [u64, u64, u32]),
        "or_upper_edges": (i64, [i32, i32p, i32p, i32p, i32p]),
        "or_exact_pairs": (None, [i32, i32p, i32p, i64, i32p, i32p, u32p]),
        "or_exact_tc_listing": (u64, [i32, i32p, i32p]),
        "or_four_cliques": (u64, [i32, i32p, i32p, i32p, ctypes.c_void_p, u32, u32, u64]),
        "or_four_cliques_filters": (None, [i32, i32p, i32p, u64p, u32, u32, u64, u64p, u64p, u64p]),
        "or_bf_build": (None, [i32, i32p, i32p, u32, u32, u64, u64p, u32p]),
        "or_bf_of_set": (None, [i32, i32p, u32, u32, u64, u64p]),
        "or_bf_counts": (None, [u32, u64p, i64, i32p, i32p, u32p, u32p]),
        "or_kh_build": (None, [i32, i32p, i32p, u32, u64, u32p]),
        "or_kh_counts": (None, [u32, u32p, i64, i32p, i32p, u32p]),
        "or_1h_build": (None, [i32, i32p, i32p, u32, u64, u32p]),
        "or_1h_counts": (None, [u32, u64, u32p, i64, i32p, i32p, u32p, u32p, u32p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a, ct):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().or_threads())


def set_threads(count: int) -> None:
    """Threads of the oracle's later parallel loops (for timing on one core)."""
    _load().or_set_threads(int(count))


# ---------------------------------------------------------------- hashing

def splitmix64(key: int, i: int) -> int:
    return int(_load().or_splitmix64(key & (2**64 - 1), i))


def hash_consts(kind: int, seed: int, count: int):
    a = np.zeros(count, dtype=np.uint64)
    c = np.zeros(count, dtype=np.uint64)
    _load().or_hash_consts(kind, seed & (2**64 - 1), count, _ptr(a, ctypes.c_uint64), _ptr(c, ctypes.c_uint64))
    return a, c


def bf_index(a: int, c: int, x: int, B: int) -> int:
    return int(_load().or_bf_index(a, c, x, B))


def mh_key(a: int, c: int, x: int) -> int:
    return int(_load().or_mh_key(a, c, x))


# ---------------------------------------------------------------- exact

def upper_edges(g):
    """The m undirected edges (v, u), v < u, in CSR order (Section 2.1, |E| = m)."""
    lib = _load()
    off, adj = _i32(g.offsets), _i32(g.adj)
    m = lib.or_upper_edges(g.n, _ptr(off, ctypes.c_int32), _ptr(adj, ctypes.c_int32), None, None)
    eu = np.empty(m, dtype=np.int32)
    ev = np.empty(m, dtype=np.int32)
    lib.or_upper_edges(g.n, _ptr(off, ctypes.c_int32), _ptr(adj, ctypes.c_int32),
                       _ptr(eu, ctypes.c_int32), _ptr(ev, ctypes.c_int32))
    return eu, ev


def arcs(g):
    """All 2m arcs (v, u), u in N_v, in CSR order."""
    deg = np.diff(g.offsets)
    return np.repeat(np.arange(g.n, dtype=np.int32), deg), _i32(g.adj)


def exact_pairs(g, u, v) -> np.ndarray:
    """|N_u intersect N_v| by sorted merge, per pair."""
    u, v = _i32(u), _i32(v)
    out = np.empty(u.shape[0], dtype=np.uint32)
    off, adj = _i32(g.offsets), _i32(g.adj)
    _load().or_exact_pairs(g.n, _ptr(off, ctypes.c_int32), _ptr(adj, ctypes.c_int32), u.shape[0],
                           _ptr(u, ctypes.c_int32), _ptr(v, ctypes.c_int32), _ptr(out, ctypes.c_uint32))
    return out


def exact_tc(g) -> int:
    """TC = (1/3) * sum over the m edges of |N_u intersect N_v| (Section 7)."""
    eu, ev = upper_edges(g)
    s = int(exact_pairs(g, eu, ev).astype(np.uint64).sum())
    assert s % 3 == 0
    return s // 3


def exact_tc_listing(g) -> int:
    """TC by the degree-ordered node iterator of Listing "lst:tc"."""
    off, adj = _i32(g.offsets), _i32(g.adj)
    return int(_load().or_exact_tc_listing(g.n, _ptr(off, ctypes.c_int32), _ptr(adj, ctypes.c_int32)))


def local_cc_from_arc_values(g, arc_values: np.ndarray) -> np.ndarray:
    """cc_v = sum_{u in N_v} I(u, v) / (d_v (d_v - 1)); 0 when d_v < 2.

    Local clustering coefficient (Watts and Strogatz 1998); sum_{u in N_v}
    |N_u cap N_v| is twice the number of triangles at v. ``arc_values`` holds
    I(v, u) for the arcs in CSR order."""
    deg = np.diff(g.offsets).astype(np.float64)
    sums = np.zeros(g.n, dtype=np.float64)
    src = np.repeat(np.arange(g.n), np.diff(g.offsets))
    np.add.at(sums, src, arc_values.astype(np.float64))
    denom = deg * (deg - 1.0)
    out = np.zeros(g.n, dtype=np.float64)
    ok = deg >= 2
    out[ok] = sums[ok] / denom[ok]
    return out


def exact_cc(g) -> np.ndarray:
    au, av = arcs(g)
    return local_cc_from_arc_values(g, exact_pairs(g, au, av))


def jaccard_from_intersection(du, dv, inter) -> np.ndarray:
    """J = |A cap B| / (|A| + |B| - |A cap B|) (Listing "lst:sim"); 0 when the union is empty.
    The intersection estimate is clamped to [0, min(d_u, d_v)] first (an estimate
    outside that range has no consistent Jaccard value)."""
    du = np.asarray(du, dtype=np.float64)
    dv = np.asarray(dv, dtype=np.float64)
    ic = np.clip(np.asarray(inter, dtype=np.float64), 0.0, np.minimum(du, dv))
    den = du + dv - ic
    out = np.zeros_like(den)
    ok = den > 0
    out[ok] = ic[ok] / den[ok]
    return out


def exact_jaccard(g, u, v) -> np.ndarray:
    deg = g.degrees()
    return jaccard_from_intersection(deg[u], deg[v], exact_pairs(g, u, v))


# ---------------------------------------------------------------- estimators

def est_bf_and(c, B: int, b: int) -> np.ndarray:
    """AND estimator, Eq. "bf_int": -(B/b) ln(1 - c~/B), c the ones of B_u AND B_v,
    with c~ = c - [c == B] so the logarithm stays finite (Appendix C)."""
    c = np.asarray(c, dtype=np.float64)
    ct = c - (c == B)
    return -(B / b) * np.log(1.0 - ct / B)


def est_bf_limit(c, B: int, b: int) -> np.ndarray:
    """Limit estimator, Eq. "limit_xs": c / b."""
    return np.asarray(c, dtype=np.float64) / b


def est_bf_papapetrou(c, B: int, b: int) -> np.ndarray:
    """Existing BF cardinality estimator (Section 8.1) applied to the AND:
    ln(1 - c~/B) / (b ln(1 - 1/B)). The paper prints a leading minus, which
    would make every estimate negative (both logarithms are negative); the
    estimator is the ratio of the two logarithms."""
    c = np.asarray(c, dtype=np.float64)
    ct = c - (c == B)
    return np.log(1.0 - ct / B) / (b * np.log(1.0 - 1.0 / B))


def est_bf_or(c_or, du, dv, B: int, b: int) -> np.ndarray:
    """OR estimator, Eq. "bf_int_union": |X| + |Y| + (B/b) ln(1 - c~_or/B)."""
    c_or = np.asarray(c_or, dtype=np.float64)
    ct = c_or - (c_or == B)
    return (np.asarray(du, np.float64) + np.asarray(dv, np.float64)) + (B / b) * np.log(1.0 - ct / B)


def est_minhash(s, kk, du, dv) -> np.ndarray:
    """MinHash intersection estimators, Eq. "est_int_mh" and Section 4.4:
    J^ = s / k, I^ = J^ / (1 + J^) * (|X| + |Y|). J^ = 0 when k = 0."""
    s = np.asarray(s, dtype=np.float64)
    kk = np.asarray(kk, dtype=np.float64) * np.ones_like(s)
    jh = np.zeros_like(s)
    ok = kk > 0
    jh[ok] = s[ok] / kk[ok]
    return jh / (1.0 + jh) * (np.asarray(du, np.float64) + np.asarray(dv, np.float64))


# ---------------------------------------------------------------- sketches

@dataclass
class Sketches:
    """Per-vertex sketches of one graph plus what the estimators need."""

    g: object
    kind: int
    size: int          # B (bits) for Bloom filters, k for MinHash
    b: int             # hash functions per Bloom filter (1 for MinHash)
    seed: int
    words: np.ndarray | None = None   # uint64 [n, B/64]
    pc: np.ndarray | None = None      # uint32 [n]
    sig: np.ndarray | None = None     # uint32 [n, k]
    deg: np.ndarray = field(default=None)

    def counts(self, u, v):
        """Integer counts per pair: BF -> (c_and, c_or); k-hash -> s;
        1-hash -> (s_union, kprime, s_literal)."""
        lib = _load()
        u, v = _i32(u), _i32(v)
        npairs = u.shape[0]
        pu, pv = _ptr(u, ctypes.c_int32), _ptr(v, ctypes.c_int32)
        if self.kind == KIND_BF:
            ca = np.empty(npairs, np.uint32)
            co = np.empty(npairs, np.uint32)
            lib.or_bf_counts(self.size // 64, _ptr(self.words, ctypes.c_uint64), npairs, pu, pv,
                             _ptr(ca, ctypes.c_uint32), _ptr(co, ctypes.c_uint32))
            return ca, co
        if self.kind == KIND_KH:
            s = np.empty(npairs, np.uint32)
            lib.or_kh_counts(self.size, _ptr(self.sig, ctypes.c_uint32), npairs, pu, pv, _ptr(s, ctypes.c_uint32))
            return s
        su = np.empty(npairs, np.uint32)
        kp = np.empty(npairs, np.uint32)
        sl = np.empty(npairs, np.uint32)
        lib.or_1h_counts(self.size, self.seed & (2**64 - 1), _ptr(self.sig, ctypes.c_uint32), npairs, pu, pv,
                         _ptr(su, ctypes.c_uint32), _ptr(kp, ctypes.c_uint32), _ptr(sl, ctypes.c_uint32))
        return su, kp, sl

    def estimate(self, u, v, est: str) -> np.ndarray:
        """FP64 estimate of |N_u cap N_v| per pair."""
        u, v = _i32(u), _i32(v)
        du, dv = self.deg[u], self.deg[v]
        if self.kind == KIND_BF:
            ca, co = self.counts(u, v)
            B, b = self.size, self.b
            if est == "and":
                return est_bf_and(ca, B, b)
            if est == "l":
                return est_bf_limit(ca, B, b)
            if est == "pap":
                return est_bf_papapetrou(ca, B, b)
            if est == "or":
                return est_bf_or(co, du, dv, B, b)
            raise ValueError(f"estimator {est} does not apply to Bloom filters")
        if self.kind == KIND_KH:
            if est != "kh":
                raise ValueError(f"estimator {est} does not apply to k-hash sketches")
            return est_minhash(self.counts(u, v), self.size, du, dv)
        if est == "1h":
            su, kp, _ = self.counts(u, v)
            return est_minhash(su, kp, du, dv)
        if est == "1h_lit":
            _, _, sl = self.counts(u, v)
            return est_minhash(sl, self.size, du, dv)
        if est in ("kmv", "kmv_est"):
            return self.kmv_estimate(u, v, est)
        raise ValueError(f"estimator {est} does not apply to 1-hash sketches")

    def kmv_keys(self):
        """Per row, the MinHash keys of its elements (ascending: a 1-hash row
        lists its elements in key order); empty slots are dropped."""
        cached = self.__dict__.get("_kmv_keys")
        if cached is not None:
            return cached
        a, c = hash_consts(KIND_1H, self.seed, 1)
        out = []
        for v in range(self.sig.shape[0]):
            row = self.sig[v]
            row = row[row != BOTTOM]
            out.append(mh_keys(int(a[0]), int(c[0]), row))
        self.__dict__["_kmv_keys"] = out
        return out

    def kmv_estimate(self, u, v, est: str) -> np.ndarray:
        """KMV estimate of |N_u cap N_v| from the rows' keys (Section "Beyond
        Bloom Filter and MinHash", Appendix "KMV Sketches"); parity: see
        kmv_intersection."""
        keys = self.kmv_keys()
        u, v = _i32(u), _i32(v)
        out = np.empty(u.shape[0], dtype=np.float64)
        for i in range(u.shape[0]):
            out[i] = kmv_intersection(keys[u[i]], keys[v[i]], self.size, int(self.deg[u[i]]),
                                      int(self.deg[v[i]]), est == "kmv")
        return out


def build_sketches(g, kind: int, size: int, b: int = 1, seed: int = 1) -> Sketches:
    lib = _load()
    off, adj = _i32(g.offsets), _i32(g.adj)
    po, pa = _ptr(off, ctypes.c_int32), _ptr(adj, ctypes.c_int32)
    sk = Sketches(g, kind, size, b if kind == KIND_BF else 1, seed, deg=g.degrees())
    s64 = seed & (2**64 - 1)
    if kind == KIND_BF:
        if size % 64 or size <= 0:
            raise ValueError("Bloom-filter size must be a positive multiple of 64 bits")
        sk.words = np.zeros((g.n, size // 64), dtype=np.uint64)
        sk.pc = np.zeros(g.n, dtype=np.uint32)
        lib.or_bf_build(g.n, po, pa, size, b, s64, _ptr(sk.words, ctypes.c_uint64), _ptr(sk.pc, ctypes.c_uint32))
    elif kind == KIND_KH:
        sk.sig = np.zeros((g.n, size), dtype=np.uint32)
        lib.or_kh_build(g.n, po, pa, size, s64, _ptr(sk.sig, ctypes.c_uint32))
    elif kind == KIND_1H:
        sk.sig = np.zeros((g.n, size), dtype=np.uint32)
        lib.or_1h_build(g.n, po, pa, size, s64, _ptr(sk.sig, ctypes.c_uint32))
    else:
        raise ValueError("unknown sketch kind")
    return sk


def bf_of_set(xs, B: int, b: int, seed: int) -> np.ndarray:
    xs = _i32(xs)
    w = np.zeros(B // 64, dtype=np.uint64)
    _load().or_bf_of_set(xs.shape[0], _ptr(xs, ctypes.c_int32), B, b, seed & (2**64 - 1), _ptr(w, ctypes.c_uint64))
    return w


# ---------------------------------------------------------------- algorithms

def tc(sk: Sketches, est: str) -> float:
    """TC^ = (1/3) * sum over the m edges of the estimate (Section 7)."""
    eu, ev = upper_edges(sk.g)
    return float(np.sum(sk.estimate(eu, ev, est)) / 3.0)


def cc(sk: Sketches, est: str) -> np.ndarray:
    """Estimated local clustering coefficient: the exact formula with the
    estimate in place of |N_u cap N_v| for every arc."""
    au, av = arcs(sk.g)
    return local_cc_from_arc_values(sk.g, sk.estimate(au, av, est))


def jaccard(sk: Sketches, est: str, u, v) -> np.ndarray:
    """Estimated Jaccard similarity (Listing "lst:sim") per pair."""
    u, v = _i32(u), _i32(v)
    return jaccard_from_intersection(sk.deg[u], sk.deg[v], sk.estimate(u, v, est))


# ---------------------------------------------------------------- KMV

def _mix64(z):
    """SplitMix64's output mix (Steele, Lea, Flood 2014) on uint64 arrays."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def mh_keys(a: int, c: int, xs) -> np.ndarray:
    """MinHash keys mix64(a x + c mod 2^64) of the IDs xs (the array form of mh_key)."""
    xs = np.asarray(xs, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64(np.uint64(a) * xs + np.uint64(c))


def kmv_hash(keys) -> np.ndarray:
    """The KMV hash h: X -> (0, 1] (Section "Beyond Bloom Filter and MinHash"):
    the top 53 bits of the MinHash key, plus one, times 2^-53."""
    k = np.asarray(keys, dtype=np.uint64)
    return ((k >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * 2.0 ** -53


def kmv_of_set(xs, k: int, seed: int) -> np.ndarray:
    """K_X: the k smallest hashes of the elements of X (all when |X| <= k), ascending."""
    a, c = hash_consts(KIND_1H, seed, 1)
    keys = np.sort(mh_keys(int(a[0]), int(c[0]), np.unique(np.asarray(xs, dtype=np.int64))))
    return kmv_hash(keys[:k])


def kmv_size(kx, k: int) -> float:
    """|X|^ = (k - 1) / max K_X (Eq. "est_ss_kmv"). A KMV holding fewer than k
    values holds the whole set, and its size is that count."""
    kx = np.asarray(kx, dtype=np.float64)
    if kx.shape[0] < k:
        return float(kx.shape[0])
    return (k - 1) / float(kx[k - 1])


def kmv_intersection(kx, ky, k: int, dx: int, dy: int, exact_sizes: bool) -> float:
    """KMV estimate of |X cap Y| from the sorted keys of the two rows.

    The union sketch K_{X u Y} is the k smallest values of K_X u K_Y (values
    are the injective 64-bit keys, so equal keys are the same element), and
    |X u Y|^ = (k - 1) / max K_{X u Y}; if both rows hold fewer than k values
    they hold the whole sets, and the union is counted. Then
    |X cap Y|^ = |X| + |Y| - |X u Y|^ with the exact sizes d_X, d_Y
    (Eq. "est_inter_set_kmv_exactsets", exact_sizes=True) or with the KMV size
    estimates (Eq. "est_inter_set_kmv"). An empty set gives 0."""
    if dx == 0 or dy == 0:
        return 0.0
    kx = np.asarray(kx, dtype=np.uint64)
    ky = np.asarray(ky, dtype=np.uint64)
    union = np.union1d(kx, ky)
    if kx.shape[0] < k and ky.shape[0] < k:
        u_hat = float(union.shape[0])
    else:
        u_hat = (k - 1) / float(kmv_hash(union[k - 1:k])[0])
    if exact_sizes:
        return (float(dx) + float(dy)) - u_hat
    return (kmv_size(kmv_hash(kx), k) + kmv_size(kmv_hash(ky), k)) - u_hat


# ---------------------------------------------------------------- oriented sketches

def oriented(g):
    """The degree-oriented neighbourhoods of Listing "lst:tc": with the order R
    that ranks vertices by (degree, ID) ascending, N+_v = {u in N_v : R(v) < R(u)},
    each list ascending by ID. Returned as a CSR over the same n vertices (m arcs
    in all) that the sketch builders take like any graph; ``degrees()`` gives d+."""
    import types
    deg = np.diff(g.offsets).astype(np.int64)
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    dst = np.asarray(g.adj, dtype=np.int64)
    keep = (deg[dst] > deg[src]) | ((deg[dst] == deg[src]) & (dst > src))
    lens = np.bincount(src[keep], minlength=g.n).astype(np.int64)
    off = np.zeros(g.n + 1, dtype=np.int32)
    off[1:] = np.cumsum(lens)
    adj = dst[keep].astype(np.int32)  # CSR order: by source, then ascending ID
    return types.SimpleNamespace(n=g.n, offsets=off, adj=adj, nnz=int(adj.shape[0]),
                                 degrees=lambda: lens.copy(), name=f"{getattr(g, 'name', '')}+")


def four_cliques(g) -> int:
    """Exact number of 4-cliques by the reformulated listing (Listing
    "lst:fcl"): for every u and v in N+_u, C3 = N+_u cap N+_v, and for every w
    in C3 add |N+_w cap C3| (each 4-clique once, at its three lowest-ranked
    vertices)."""
    o = oriented(g)
    deg = _i32(np.diff(g.offsets))
    po, pa = _i32(o.offsets), _i32(o.adj)
    return int(_load().or_four_cliques(g.n, _ptr(po, ctypes.c_int32), _ptr(pa, ctypes.c_int32),
                                       _ptr(deg, ctypes.c_int32), None, 64, 1, 0))


def four_cliques_bf(g, sk_plus: Sketches) -> int:
    """4-cliques with |N+_w cap C3| estimated from the Bloom filter of N+_w
    (``sk_plus``: filters of the oriented sets): the number of x in C3 ranked
    above w (the only elements N+_w can hold) that pass the membership query of
    the filter. Membership queries have false positives only, so the estimate
    is never below the exact count."""
    assert sk_plus.kind == KIND_BF
    o = oriented(g)
    deg = _i32(np.diff(g.offsets))
    po, pa = _i32(o.offsets), _i32(o.adj)
    words = np.ascontiguousarray(sk_plus.words)
    return int(_load().or_four_cliques(g.n, _ptr(po, ctypes.c_int32), _ptr(pa, ctypes.c_int32),
                                       _ptr(deg, ctypes.c_int32), words.ctypes.data_as(ctypes.c_void_p),
                                       sk_plus.size, sk_plus.b, sk_plus.seed & (2**64 - 1)))


def four_cliques_filter_counts(g, sk_plus: Sketches):
    """For every oriented edge (u, v) and every w in C3 = N+_u cap N+_v, the
    ones c of (filter of N+_w) AND (filter of C3) and c_or of their OR, the
    filter of C3 built with the hash functions of ``sk_plus`` (filters of the
    oriented sets). Returns (hist_and, hist_or, sizes): how often each value
    of c and of c_or occurs (B + 1 entries each) and the sum of |N+_w| + |C3|
    over all (edge, w)."""
    assert sk_plus.kind == KIND_BF
    o = oriented(g)
    po, pa = _i32(o.offsets), _i32(o.adj)
    words = np.ascontiguousarray(sk_plus.words, dtype=np.uint64)
    B = sk_plus.size
    ha = np.zeros(B + 1, np.uint64)
    ho = np.zeros(B + 1, np.uint64)
    sizes = ctypes.c_uint64(0)
    _load().or_four_cliques_filters(g.n, _ptr(po, ctypes.c_int32), _ptr(pa, ctypes.c_int32),
                                    _ptr(words, ctypes.c_uint64), B, sk_plus.b, sk_plus.seed & (2**64 - 1),
                                    _ptr(ha, ctypes.c_uint64), _ptr(ho, ctypes.c_uint64), ctypes.byref(sizes))
    return ha, ho, int(sizes.value)


def four_cliques_estimate(g, sk_plus: Sketches, est: str) -> float:
    """4-cliques with |N+_w cap C3| estimated by a Bloom-filter estimator of
    the intersection of N+_w and C3 (Listing "lst:fcl" with sketch
    intersections): the sum over all (edge, w) of the estimate, formed as the
    count of each value of c (or c_or) times the estimator at that value, plus
    the exact integer sum of |N+_w| + |C3| for the OR estimator."""
    ha, ho, sizes = four_cliques_filter_counts(g, sk_plus)
    B, b = sk_plus.size, sk_plus.b
    c = np.arange(B + 1)
    if est == "and":
        t = est_bf_and(c, B, b)
    elif est == "l":
        t = est_bf_limit(c, B, b)
    elif est == "pap":
        t = est_bf_papapetrou(c, B, b)
    elif est == "or":
        return float(sizes) + float(np.sum(ho.astype(np.float64) * est_bf_or(c, 0, 0, B, b)))
    else:
        raise ValueError(f"estimator {est} does not apply to Bloom filters")
    return float(np.sum(ha.astype(np.float64) * t))


def tc_oriented(g, sk_plus: Sketches, est: str) -> float:
    """TC^ from sketches of the oriented sets (Listing "lst:tc"): the sum over
    the oriented edges (v, u), u in N+_v, of the estimate of |N+_v cap N+_u|,
    with no factor 1/3 (a triangle a, b, c with R(a) < R(b) < R(c) lies in
    N+_a cap N+_b only). The intersection is symmetric in its two sets, so the
    sum runs over the m undirected edges of g, each once."""
    eu, ev = upper_edges(g)
    return float(np.sum(sk_plus.estimate(eu, ev, est)))


# ---------------------------------------------------------------- similarity and clustering

SIM_COMMON, SIM_JACCARD, SIM_OVERLAP, SIM_TOTAL = 0, 1, 2, 3
SIMILARITIES = {"cn": SIM_COMMON, "jaccard": SIM_JACCARD, "overlap": SIM_OVERLAP, "total": SIM_TOTAL}


def similarity_from_intersection(du, dv, inter, measure: int) -> np.ndarray:
    """Vertex similarity of two neighbourhoods A = N_u, B = N_v from |A cap B|
    (Listing "lst:sim"):

    * common neighbours: |A cap B| itself (an estimate is passed on as it is);
    * Jaccard: |A cap B| / (|A| + |B| - |A cap B|), 0 when the union is empty;
    * overlap: |A cap B| / min(|A|, |B|), 0 when the smaller set is empty;
    * total neighbours: |A cup B| = |A| + |B| - |A cap B|.

    For Jaccard, overlap and total neighbours an estimate is clamped to
    [0, min(d_u, d_v)] first, the range of a true intersection (no other value
    gives a consistent union)."""
    inter = np.asarray(inter, dtype=np.float64)
    if measure == SIM_COMMON:
        return inter.copy()
    if measure == SIM_JACCARD:
        return jaccard_from_intersection(du, dv, inter)
    du = np.asarray(du, dtype=np.float64)
    dv = np.asarray(dv, dtype=np.float64)
    lo = np.minimum(du, dv)
    ic = np.clip(inter, 0.0, lo)
    if measure == SIM_OVERLAP:
        out = np.zeros_like(ic)
        ok = lo > 0
        out[ok] = ic[ok] / lo[ok]
        return out
    if measure == SIM_TOTAL:
        return (du + dv) - ic
    raise ValueError(f"unknown similarity measure {measure}")


def exact_similarity(g, u, v, measure: int) -> np.ndarray:
    """Exact vertex similarity per pair (exact intersections by merge)."""
    deg = g.degrees()
    u, v = _i32(u), _i32(v)
    return similarity_from_intersection(deg[u], deg[v], exact_pairs(g, u, v), measure)


def similarity(sk: Sketches, est: str, u, v, measure: int) -> np.ndarray:
    """Estimated vertex similarity per pair: the estimate of |N_u cap N_v| in
    place of the exact intersection."""
    u, v = _i32(u), _i32(v)
    return similarity_from_intersection(sk.deg[u], sk.deg[v], sk.estimate(u, v, est), measure)


def jarvis_patrick(values, tau: float) -> np.ndarray:
    """Jarvis-Patrick clustering (Listing "lst:cl"): an edge belongs to the
    clustering C when the similarity of its endpoints is greater than the
    threshold tau. ``values`` holds the similarity of the m upper edges;
    returns C as a 0/1 uint8 mask over them."""
    return (np.asarray(values, dtype=np.float64) > tau).astype(np.uint8)


def exact_jarvis_patrick(g, measure: int, tau: float) -> np.ndarray:
    eu, ev = upper_edges(g)
    return jarvis_patrick(exact_similarity(g, eu, ev, measure), tau)


def estimated_jarvis_patrick(sk: Sketches, est: str, measure: int, tau: float) -> np.ndarray:
    eu, ev = upper_edges(sk.g)
    return jarvis_patrick(similarity(sk, est, eu, ev, measure), tau)


def clusters(n: int, eu, ev, keep=None) -> np.ndarray:
    """The clusters of an edge set C: the connected components of (V, C), every
    vertex labelled with the smallest vertex ID of its component (a vertex
    without an edge in C is a cluster of its own). ``keep`` selects C among the
    edges (eu, ev); None takes them all.

    label_v is the smallest ID reachable from v; it is reached by repeating
    label_v <- min(label_v, label_u) over the edges of C (both directions)
    until no label changes."""
    eu = np.asarray(eu, dtype=np.int64)
    ev = np.asarray(ev, dtype=np.int64)
    if keep is not None:
        sel = np.asarray(keep).astype(bool)
        eu, ev = eu[sel], ev[sel]
    label = np.arange(n, dtype=np.int64)
    while True:
        low = np.minimum(label[eu], label[ev])
        new = label.copy()
        np.minimum.at(new, eu, low)
        np.minimum.at(new, ev, low)
        if np.array_equal(new, label):
            return label.astype(np.int32)
        label = new


def cluster_count(labels) -> int:
    """Number of clusters: the vertices that label themselves."""
    labels = np.asarray(labels)
    return int(np.count_nonzero(labels == np.arange(labels.shape[0])))


def bits_for_budget(g, s: float) -> int:
    """Bloom-filter size for storage budget s (Section 5.1): the largest
    multiple of 64 bits with n * B <= s * 8 * CSR bytes, at least 64."""
    csr_bytes = 4 * (g.n + 1) + 4 * g.nnz
    return max(64, 64 * int(s * 8 * csr_bytes // (64 * g.n)))


def sketch_rows(g, verts, kind: int, size: int, b: int = 1, seed: int = 1) -> Sketches:
    """Sketches of the listed vertices only: row i is the sketch of N_{verts[i]},
    by the same definition as ``build_sketches`` (used to check samples of a
    large graph). ``deg`` holds the degrees of the listed vertices."""
    import types
    verts = np.asarray(verts, dtype=np.int64)
    lens = g.degrees()[verts]
    off = np.zeros(len(verts) + 1, dtype=np.int32)
    off[1:] = np.cumsum(lens)
    parts = [g.adj[g.offsets[v]:g.offsets[v + 1]] for v in verts]
    adj = np.concatenate(parts).astype(np.int32) if parts else np.zeros(0, np.int32)
    sub = types.SimpleNamespace(n=len(verts), offsets=off, adj=adj, nnz=int(adj.shape[0]),
                                degrees=lambda: lens.astype(np.int64))
    return build_sketches(sub, kind, size, b, seed)
