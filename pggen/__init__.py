"""Seeded synthetic inputs: CSR graphs, graph batches and pair-query traces.

Inputs only: nothing here computes a sketch, a hash of the method or an
estimate. The test oracle and the GPU library are both fed from these arrays.

Graph layout (Section 2.1 of the paper): ``offsets`` int32[n+1] and ``adj``
int32[nnz]; each neighbourhood N_v = adj[offsets[v]:offsets[v+1]] is sorted
ascending, symmetric (u in N_v iff v in N_u), without duplicates or self-loops.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pggen.cpp")
_LIB_PATH = os.path.join(_HERE, "libpggen.so")
_lib = None


def build() -> str:
    """Compile the generator's shared library (g++, OpenMP)."""
    tmp = _LIB_PATH + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp]
    subprocess.check_call(cmd)
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
    lib.pggen_splitmix64.restype = ctypes.c_uint64
    lib.pggen_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.pggen_rmat_pairs.restype = ctypes.c_int
    lib.pggen_rmat_pairs.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_uint64, i32p, i32p]
    lib.pggen_er_pairs.restype = ctypes.c_int64
    lib.pggen_er_pairs.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, i32p, i32p,
                                   ctypes.c_int64]
    lib.pggen_csr_build.restype = ctypes.c_int64
    lib.pggen_csr_build.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, i32p, i32p,
                                    ctypes.c_int64]
    _lib = lib
    return lib


def _p32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


@dataclass
class CSR:
    """An undirected graph in CSR form (int32 offsets and neighbour IDs)."""

    n: int
    offsets: np.ndarray
    adj: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.adj.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.offsets).astype(np.int64)

    def neighbours(self, v: int) -> np.ndarray:
        return self.adj[self.offsets[v]:self.offsets[v + 1]]

    def csr_bytes(self) -> int:
        return 4 * (self.n + 1) + 4 * self.nnz


def splitmix64(key: int, i: int) -> int:
    """Output i (0-based) of the SplitMix64 stream with initial state ``key``."""
    return int(_load().pggen_splitmix64(ctypes.c_uint64(key & (2**64 - 1)), ctypes.c_uint64(i)))


def from_pairs(n: int, src, dst, name: str = "") -> CSR:
    """Symmetric, sorted, deduplicated CSR from (src, dst) pairs; self-loops dropped."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    assert src.shape == dst.shape
    lib = _load()
    cap = 2 * int(src.shape[0])
    offsets = np.zeros(n + 1, dtype=np.int32)
    adj = np.empty(max(cap, 1), dtype=np.int32)
    nnz = lib.pggen_csr_build(n, int(src.shape[0]), _p32(src), _p32(dst), _p32(offsets), _p32(adj), cap)
    if nnz < 0:
        raise ValueError(f"pggen_csr_build failed ({nnz})")
    return CSR(n, offsets, adj[:nnz].copy(), name)


def rmat(scale: int, edge_factor: int, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1, n: int | None = None) -> CSR:
    """R-MAT graph with 2**scale vertices (or ``n`` vertices with rejection) and
    edge_factor * n draws, symmetrized, deduplicated, without self-loops."""
    if n is None:
        n = 1 << scale
    npairs = int(edge_factor) * int(n)
    src = np.empty(npairs, dtype=np.int32)
    dst = np.empty(npairs, dtype=np.int32)
    rc = _load().pggen_rmat_pairs(n, npairs, a, b, c, ctypes.c_uint64(seed), _p32(src), _p32(dst))
    if rc != 0:
        raise ValueError("bad R-MAT parameters")
    g = from_pairs(n, src, dst, name=f"rmat-n{n}-ef{edge_factor}-seed{seed}")
    return g


def er(n: int, avg_degree: float, seed: int = 1) -> CSR:
    """Erdos-Renyi G(n, p) with p = avg_degree / (n - 1)."""
    p = min(1.0, avg_degree / max(n - 1, 1))
    lib = _load()
    cnt = lib.pggen_er_pairs(n, p, ctypes.c_uint64(seed), None, None, 0)
    if cnt < 0:
        raise ValueError("bad G(n,p) parameters")
    src = np.empty(max(cnt, 1), dtype=np.int32)
    dst = np.empty(max(cnt, 1), dtype=np.int32)
    cnt2 = lib.pggen_er_pairs(n, p, ctypes.c_uint64(seed), _p32(src), _p32(dst), cnt)
    assert cnt2 == cnt
    return from_pairs(n, src[:cnt], dst[:cnt], name=f"er-n{n}-d{avg_degree}-seed{seed}")


# ---- small graph families with known structure -------------------------------------------

def complete(n: int) -> CSR:
    s, d = np.triu_indices(n, 1)
    return from_pairs(n, s, d, name=f"K{n}")


def star(leaves: int) -> CSR:
    return from_pairs(leaves + 1, np.zeros(leaves, np.int32), np.arange(1, leaves + 1), name=f"S{leaves}")


def cycle(n: int) -> CSR:
    v = np.arange(n)
    return from_pairs(n, v, (v + 1) % n, name=f"C{n}")


def wheel(rim: int) -> CSR:
    """Hub 0 joined to a cycle 1..rim."""
    v = np.arange(1, rim + 1)
    src = np.concatenate([np.zeros(rim, np.int64), v])
    dst = np.concatenate([v, (v % rim) + 1])
    return from_pairs(rim + 1, src, dst, name=f"W{rim}")


def complete_bipartite(a: int, b: int) -> CSR:
    s, d = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return from_pairs(a + b, s.ravel(), d.ravel(), name=f"K{a},{b}")


def friendship(k: int) -> CSR:
    """k triangles sharing the hub 0."""
    src, dst = [], []
    for i in range(k):
        x, y = 1 + 2 * i, 2 + 2 * i
        src += [0, 0, x]
        dst += [x, y, y]
    return from_pairs(2 * k + 1, src, dst, name=f"F{k}")


def disjoint_union(*gs: CSR) -> CSR:
    src, dst, base = [], [], 0
    for g in gs:
        deg = np.diff(g.offsets)
        s = np.repeat(np.arange(g.n), deg)
        src.append(s + base)
        dst.append(g.adj.astype(np.int64) + base)
        base += g.n
    return from_pairs(base, np.concatenate(src), np.concatenate(dst), name="+".join(g.name for g in gs))


def from_adjacency_bits(n: int, bits: int) -> CSR:
    """Graph on n vertices whose edge set is the bitmask over the pairs i<j in
    lexicographic order (used to enumerate every graph on a few vertices)."""
    s, d = np.triu_indices(n, 1)
    sel = np.array([(bits >> i) & 1 for i in range(s.shape[0])], dtype=bool)
    return from_pairs(n, s[sel], d[sel], name=f"g{n}-{bits}")


# ---- batches and query traces --------------------------------------------------------------

def graph_batch(count: int = 512, seed0: int = 1, log2_lo: float = 8.0, log2_hi: float = 16.0):
    """A batch of independent graphs of uneven size: n_g = floor(2**U), U ~ U[lo, hi];
    even g are G(n, p) with mean degree drawn from {8..64}, odd g are R-MAT with
    edge factor 16 on n_g vertices; per-graph Bloom-filter size drawn from
    {128, 192, ..., 1024} bits. Returns (graphs, bf_bits)."""
    graphs, bits = [], []
    for g in range(count):
        rng = np.random.default_rng(seed0 + g)
        n_g = int(math.floor(2.0 ** rng.uniform(log2_lo, log2_hi)))
        b_g = int(64 * rng.integers(2, 17))
        if g % 2 == 0:
            deg = int(rng.integers(8, 65))
            graphs.append(er(n_g, deg, seed=seed0 + g))
        else:
            graphs.append(rmat(0, 16, seed=seed0 + g, n=n_g))
        bits.append(b_g)
    return graphs, bits


@dataclass
class Request:
    arrival_s: float
    op: str          # "cn" (common-neighbour estimate) or "jaccard"
    kind: str        # "bf" or "mh"
    u: np.ndarray    # int32[L]
    v: np.ndarray    # int32[L]


def query_trace(n: int, count: int, rate_hz: float, seed: int = 1, log2_max: float = 16.0):
    """Poisson arrivals; each request is L = floor(2**U), U ~ U[0, log2_max], uniformly random
    vertex pairs with u != v; op and sketch kind uniform."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += rng.exponential(1.0 / rate_hz) if rate_hz > 0 else 0.0
        L = int(math.floor(2.0 ** rng.uniform(0.0, log2_max)))
        u = rng.integers(0, n, size=L, dtype=np.int64)
        v = rng.integers(0, n - 1, size=L, dtype=np.int64)
        v = np.where(v >= u, v + 1, v)
        op = "cn" if rng.integers(0, 2) == 0 else "jaccard"
        kind = "bf" if rng.integers(0, 2) == 0 else "mh"
        out.append(Request(t, op, kind, u.astype(np.int32), v.astype(np.int32)))
    return out
