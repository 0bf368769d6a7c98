"""ProbGraph on MI355X: a thin ctypes binding over ``libprobgraph.so``.

The functions named ``pg_*`` mirror the C ABI in ``include/probgraph.h`` one to
one (argument marshalling only: every step runs in the library's HIP kernels).
``Context``, ``Graph`` and ``Sketches`` wrap the handles for convenience.
Device buffers are torch tensors on the context's GPU; streams default to
torch's current stream. There is no CPU fallback: if the library is not built
or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libprobgraph.so")

# return codes
PG_OK = 0
PG_E_INVALID = -1
PG_E_GRAPH = -2
PG_E_NOMEM = -3
PG_E_DEVICE = -4
PG_E_UNSUPPORTED = -5
PG_E_BUSY = -6
# sketch kinds
PG_BF = 1
PG_MH_KHASH = 2
PG_MH_1HASH = 3
PG_ORIENTED = 256  # flag: sketch the degree-oriented sets N+_v
# estimators
PG_EST_BF_AND = 1
PG_EST_BF_L = 2
PG_EST_BF_OR = 3
PG_EST_BF_PAPAPETROU = 4
PG_EST_MH_KHASH = 5
PG_EST_MH_1HASH = 6
PG_EST_MH_1HASH_LITERAL = 7
PG_EST_KMV = 8
PG_EST_KMV_SKETCH_SIZES = 9
# graph flags
PG_MEM_HOST = 0
PG_MEM_DEVICE = 1
PG_BORROW = 2
PG_VALIDATE = 4
# exact algorithms
PG_EXACT_MERGE = 1
PG_EXACT_BITMAP = 2
# similarity measures (Listing "lst:sim")
PG_SIM_COMMON = 0
PG_SIM_JACCARD = 1
PG_SIM_OVERLAP = 2
PG_SIM_TOTAL = 3

ESTIMATORS = {
    "and": PG_EST_BF_AND, "l": PG_EST_BF_L, "or": PG_EST_BF_OR, "pap": PG_EST_BF_PAPAPETROU,
    "kh": PG_EST_MH_KHASH, "1h": PG_EST_MH_1HASH, "1h_lit": PG_EST_MH_1HASH_LITERAL,
    "kmv": PG_EST_KMV, "kmv_est": PG_EST_KMV_SKETCH_SIZES,
}
KINDS = {"bf": PG_BF, "kh": PG_MH_KHASH, "1h": PG_MH_1HASH}
SKETCH_FILE_FORMAT = "probgraph-sketches-1"
HASH_FAMILY = "splitmix64-affine-1"  # the seeded hash family of pg_build_sketches (see probgraph.h)
SIMILARITIES = {"cn": PG_SIM_COMMON, "jaccard": PG_SIM_JACCARD, "overlap": PG_SIM_OVERLAP, "total": PG_SIM_TOTAL}


class PGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"probgraph error {code}: {msg}")
        self.code = code


class _GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("max_degree", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("m", ctypes.c_int64)]


class _KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


class _SketchInfo(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("size", ctypes.c_uint32), ("b", ctypes.c_uint32),
                ("row_bytes", ctypes.c_uint32), ("seed", ctypes.c_uint64), ("total_bytes", ctypes.c_uint64)]


class _BatchParams(ctypes.Structure):
    _fields_ = [("tile_vertices", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32)]


class _ServerParams(ctypes.Structure):
    _fields_ = [("max_batches_in_flight", ctypes.c_int32), ("max_pairs_per_request", ctypes.c_int32),
                ("max_batch_pairs", ctypes.c_int64), ("memory_budget_bytes", ctypes.c_uint64)]


class _Request(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("sketch", ctypes.c_int32), ("estimator", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("npairs", ctypes.c_int64), ("u", ctypes.c_void_p),
                ("v", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("rejected_busy", ctypes.c_uint64),
                ("rejected_invalid", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("pairs", ctypes.c_uint64), ("max_in_flight", ctypes.c_uint64),
                ("max_batch_requests", ctypes.c_uint64)]


PG_OP_CN = 1
PG_OP_JACCARD = 2

_lib = None
_vp = ctypes.c_void_p


def _declare(lib):
    P = ctypes.POINTER
    i32, i64, u32, u64, i = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    sigs = {
        "pg_last_error": (ctypes.c_char_p, []),
        "pg_version": (ctypes.c_char_p, []),
        "pg_ctx_create": (i, [i, P(_vp)]),
        "pg_ctx_destroy": (i, [_vp]),
        "pg_graph_create": (i, [_vp, i32, i64, _vp, _vp, u32, _vp, P(_vp)]),
        "pg_graph_destroy": (i, [_vp]),
        "pg_graph_get_info": (i, [_vp, P(_GraphInfo)]),
        "pg_graph_upper_edges": (i, [_vp, _vp, _vp, _vp]),
        "pg_sketch_bits_for_budget": (i, [_vp, ctypes.c_double, P(u32)]),
        "pg_build_sketches": (i, [_vp, _vp, i, u32, u32, u64, _vp, P(_vp)]),
        "pg_sketches_destroy": (i, [_vp]),
        "pg_sketches_get_info": (i, [_vp, P(_SketchInfo)]),
        "pg_sketches_export": (i, [_vp, _vp, _vp, _vp]),
        "pg_sketches_import": (i, [_vp, _vp, i, u32, u32, u64, _vp, _vp, _vp, P(_vp)]),
        "pg_intersect_edges": (i, [_vp, _vp, i, _vp, _vp, i64, _vp, _vp, _vp]),
        "pg_tc": (i, [_vp, _vp, i, P(ctypes.c_double), _vp]),
        "pg_tc_async": (i, [_vp, _vp, i, _vp, _vp]),
        "pg_tc_noalloc": (i, [_vp, _vp, i, _vp, _vp]),
        "pg_cc": (i, [_vp, _vp, i, _vp, P(ctypes.c_double), _vp]),
        "pg_jaccard": (i, [_vp, _vp, i, _vp, _vp, i64, _vp, _vp]),
        "pg_exact_intersect_edges": (i, [_vp, _vp, i, _vp, _vp, i64, _vp, _vp]),
        "pg_exact_tc": (i, [_vp, _vp, i, P(u64), _vp]),
        "pg_exact_cc": (i, [_vp, _vp, _vp, P(ctypes.c_double), _vp]),
        "pg_exact_jaccard": (i, [_vp, _vp, _vp, _vp, i64, _vp, _vp]),
        "pg_similarity": (i, [_vp, _vp, i, i, _vp, _vp, i64, _vp, _vp]),
        "pg_exact_similarity": (i, [_vp, _vp, i, _vp, _vp, i64, _vp, _vp]),
        "pg_jarvis_patrick": (i, [_vp, _vp, i, i, ctypes.c_double, _vp, P(i64), _vp]),
        "pg_exact_jarvis_patrick": (i, [_vp, _vp, i, i, ctypes.c_double, _vp, P(i64), _vp]),
        "pg_clusters": (i, [_vp, _vp, _vp, _vp, P(i64), _vp]),
        "pg_exact_four_cliques": (i, [_vp, _vp, P(u64), _vp]),
        "pg_four_cliques": (i, [_vp, _vp, P(u64), _vp]),
        "pg_four_cliques_estimate": (i, [_vp, _vp, i, P(ctypes.c_double), _vp]),
        "pg_sketches_rebuild": (i, [_vp, _vp, u64, _vp]),
        "pg_profile_enable": (i, [_vp, i]),
        "pg_profile_select": (i, [_vp, ctypes.c_char_p]),
        "pg_profile_read": (i, [_vp, P(_KernelTime), i, P(i)]),
        "pg_profile_reset": (i, [_vp]),
        "pg_copy": (i, [_vp, _vp, _vp, ctypes.c_size_t, _vp]),
        "pg_server_create": (i, [_vp, _vp, P(_vp), i32, P(_ServerParams), P(_vp)]),
        "pg_server_submit": (i, [_vp, P(_Request), P(u64)]),
        "pg_server_poll": (i, [_vp, u64, P(i32)]),
        "pg_server_wait": (i, [_vp, u64, P(ctypes.c_double)]),
        "pg_server_get_stats": (i, [_vp, P(_ServerStats)]),
        "pg_server_replay": (i, [_vp, i64, P(_Request), P(ctypes.c_double), i32, P(ctypes.c_double),
                                 P(ctypes.c_double)]),
        "pg_server_destroy": (i, [_vp]),
        "pg_batch_create": (i, [_vp, i32, P(_vp), P(_vp), P(i32), P(i64), P(u32), u32, u64, P(_vp)]),
        "pg_batch_set_params": (i, [_vp, P(_BatchParams)]),
        "pg_batch_get_params": (i, [_vp, P(_BatchParams)]),
        "pg_batch_run": (i, [_vp, i, _vp]),
        "pg_batch_capture": (i, [_vp, i, _vp]),
        "pg_batch_replay": (i, [_vp, _vp]),
        "pg_batch_results": (i, [_vp, P(ctypes.c_double), P(ctypes.c_float), _vp]),
        "pg_batch_autotune": (i, [_vp, i, _vp, P(ctypes.c_double)]),
        "pg_batch_destroy": (i, [_vp]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return list(sigs)


EXPORTED = None


def load():
    """Load the built library (raises if it was not built)."""
    global _lib, EXPORTED
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2208_11469_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    EXPORTED = _declare(lib)
    _lib = lib
    return lib


def _check(rc: int):
    if rc != PG_OK:
        raise PGError(rc, load().pg_last_error().decode())


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dptr(t, dtype=None):
    """Device pointer of a contiguous CUDA tensor (or None)."""
    if t is None:
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device (cuda) tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return t.data_ptr()


# ---- the C ABI, one wrapper per call ------------------------------------------------

def pg_version() -> str:
    return load().pg_version().decode()


def pg_last_error() -> str:
    return load().pg_last_error().decode()


def pg_ctx_create(device: int = 0):
    # torch's HIP runtime first: it does not find the GPUs if the library's
    # runtime initialised them before it in this process
    _torch().cuda.init()
    h = _vp()
    _check(load().pg_ctx_create(device, ctypes.byref(h)))
    return h


def pg_ctx_destroy(ctx):
    _check(load().pg_ctx_destroy(ctx))


def pg_graph_create(ctx, n, nnz, offsets_ptr, adj_ptr, flags, stream=None):
    h = _vp()
    _check(load().pg_graph_create(ctx, n, nnz, offsets_ptr, adj_ptr, flags, _stream(stream), ctypes.byref(h)))
    return h


def pg_graph_destroy(g):
    _check(load().pg_graph_destroy(g))


def pg_graph_get_info(g) -> _GraphInfo:
    info = _GraphInfo()
    _check(load().pg_graph_get_info(g, ctypes.byref(info)))
    return info


def pg_graph_upper_edges(g, eu, ev, stream=None):
    torch = _torch()
    _check(load().pg_graph_upper_edges(g, _dptr(eu, torch.int32), _dptr(ev, torch.int32), _stream(stream)))


def pg_sketch_bits_for_budget(g, s: float) -> int:
    bits = ctypes.c_uint32()
    _check(load().pg_sketch_bits_for_budget(g, s, ctypes.byref(bits)))
    return int(bits.value)


def pg_build_sketches(ctx, g, kind, size, b, seed, stream=None):
    h = _vp()
    _check(load().pg_build_sketches(ctx, g, kind, size, b, seed & (2**64 - 1), _stream(stream), ctypes.byref(h)))
    return h


def pg_sketches_import(ctx, g, kind, size, b, seed, rows, pc=None, stream=None):
    h = _vp()
    _check(load().pg_sketches_import(ctx, g, kind, size, b, seed & (2**64 - 1), _dptr(rows), _dptr(pc),
                                     _stream(stream), ctypes.byref(h)))
    return h


def pg_sketches_destroy(sk):
    _check(load().pg_sketches_destroy(sk))


def pg_sketches_get_info(sk) -> _SketchInfo:
    info = _SketchInfo()
    _check(load().pg_sketches_get_info(sk, ctypes.byref(info)))
    return info


def pg_sketches_export(sk, rows, pc, stream=None):
    _check(load().pg_sketches_export(sk, _dptr(rows), _dptr(pc), _stream(stream)))


def pg_intersect_edges(ctx, sk, estimator, u, v, npairs, est, raw, stream=None):
    _check(load().pg_intersect_edges(ctx, sk, estimator, _dptr(u), _dptr(v), npairs, _dptr(est), _dptr(raw),
                                     _stream(stream)))


def pg_tc(ctx, sk, estimator, stream=None) -> float:
    out = ctypes.c_double()
    _check(load().pg_tc(ctx, sk, estimator, ctypes.byref(out), _stream(stream)))
    return float(out.value)


def pg_tc_async(ctx, sk, estimator, d_tc, stream=None):
    torch = _torch()
    _check(load().pg_tc_async(ctx, sk, estimator, _dptr(d_tc, torch.float64), _stream(stream)))


def pg_tc_noalloc(ctx, sk, estimator, d_tc, stream=None):
    torch = _torch()
    _check(load().pg_tc_noalloc(ctx, sk, estimator, _dptr(d_tc, torch.float64), _stream(stream)))


def pg_cc(ctx, sk, estimator, cc, want_transitivity=False, stream=None):
    t = ctypes.c_double()
    _check(load().pg_cc(ctx, sk, estimator, _dptr(cc), ctypes.byref(t) if want_transitivity else None,
                        _stream(stream)))
    return float(t.value) if want_transitivity else None


def pg_jaccard(ctx, sk, estimator, u, v, npairs, out, stream=None):
    _check(load().pg_jaccard(ctx, sk, estimator, _dptr(u), _dptr(v), npairs, _dptr(out), _stream(stream)))


def pg_exact_intersect_edges(ctx, g, algo, u, v, npairs, out, stream=None):
    _check(load().pg_exact_intersect_edges(ctx, g, algo, _dptr(u), _dptr(v), npairs, _dptr(out), _stream(stream)))


def pg_exact_tc(ctx, g, algo, stream=None) -> int:
    out = ctypes.c_uint64()
    _check(load().pg_exact_tc(ctx, g, algo, ctypes.byref(out), _stream(stream)))
    return int(out.value)


def pg_exact_cc(ctx, g, cc, want_transitivity=False, stream=None):
    t = ctypes.c_double()
    _check(load().pg_exact_cc(ctx, g, _dptr(cc), ctypes.byref(t) if want_transitivity else None, _stream(stream)))
    return float(t.value) if want_transitivity else None


def pg_exact_jaccard(ctx, g, u, v, npairs, out, stream=None):
    _check(load().pg_exact_jaccard(ctx, g, _dptr(u), _dptr(v), npairs, _dptr(out), _stream(stream)))


def pg_similarity(ctx, sk, estimator, measure, u, v, npairs, out, stream=None):
    _check(load().pg_similarity(ctx, sk, estimator, measure, _dptr(u), _dptr(v), npairs, _dptr(out),
                                _stream(stream)))


def pg_exact_similarity(ctx, g, measure, u, v, npairs, out, stream=None):
    _check(load().pg_exact_similarity(ctx, g, measure, _dptr(u), _dptr(v), npairs, _dptr(out), _stream(stream)))


def pg_jarvis_patrick(ctx, sk, estimator, measure, tau, keep, want_count=True, stream=None):
    kept = ctypes.c_int64(-1)
    _check(load().pg_jarvis_patrick(ctx, sk, estimator, measure, float(tau), _dptr(keep),
                                    ctypes.byref(kept) if want_count else None, _stream(stream)))
    return kept.value if want_count else None


def pg_exact_jarvis_patrick(ctx, g, algo, measure, tau, keep, want_count=True, stream=None):
    kept = ctypes.c_int64(-1)
    _check(load().pg_exact_jarvis_patrick(ctx, g, algo, measure, float(tau), _dptr(keep),
                                          ctypes.byref(kept) if want_count else None, _stream(stream)))
    return kept.value if want_count else None


def pg_clusters(ctx, g, keep, label, want_count=True, stream=None):
    count = ctypes.c_int64(-1)
    _check(load().pg_clusters(ctx, g, _dptr(keep), _dptr(label), ctypes.byref(count) if want_count else None,
                              _stream(stream)))
    return count.value if want_count else None


def pg_exact_four_cliques(ctx, g, stream=None) -> int:
    out = ctypes.c_uint64(0)
    _check(load().pg_exact_four_cliques(ctx, g, ctypes.byref(out), _stream(stream)))
    return out.value


def pg_four_cliques(ctx, sk, stream=None) -> int:
    out = ctypes.c_uint64(0)
    _check(load().pg_four_cliques(ctx, sk, ctypes.byref(out), _stream(stream)))
    return out.value


def pg_four_cliques_estimate(ctx, sk, estimator, stream=None) -> float:
    out = ctypes.c_double(0.0)
    _check(load().pg_four_cliques_estimate(ctx, sk, estimator, ctypes.byref(out), _stream(stream)))
    return out.value


def pg_sketches_rebuild(ctx, sk, seed, stream=None):
    _check(load().pg_sketches_rebuild(ctx, sk, seed & (2**64 - 1), _stream(stream)))


def pg_profile_enable(ctx, enable: bool):
    _check(load().pg_profile_enable(ctx, 1 if enable else 0))


def pg_profile_select(ctx, name=None):
    """Record only the launch site `name` (None: all)."""
    _check(load().pg_profile_select(ctx, name.encode() if name else None))


def pg_profile_read(ctx) -> dict:
    """{launch site: (launches, total_ms)} since the last reset (waits for the events)."""
    cap = 64
    arr = (_KernelTime * cap)()
    cnt = ctypes.c_int()
    _check(load().pg_profile_read(ctx, arr, cap, ctypes.byref(cnt)))
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(min(cnt.value, cap))}


def pg_profile_reset(ctx):
    _check(load().pg_profile_reset(ctx))


def pg_copy(ctx, dst, src, nbytes, stream=None):
    _check(load().pg_copy(ctx, _dptr(dst), _dptr(src), nbytes, _stream(stream)))


def pg_server_create(ctx, g, sketch_handles, params=None):
    arr = (_vp * len(sketch_handles))(*[h.value if isinstance(h, _vp) else h for h in sketch_handles])
    h = _vp()
    _check(load().pg_server_create(ctx, g, arr, len(sketch_handles), ctypes.byref(params) if params else None,
                                   ctypes.byref(h)))
    return h


def pg_server_submit(srv, req) -> int:
    """Returns the ticket; raises PGError (code PG_E_BUSY when not admitted)."""
    t = ctypes.c_uint64()
    _check(load().pg_server_submit(srv, ctypes.byref(req), ctypes.byref(t)))
    return int(t.value)


def pg_server_poll(srv, ticket) -> bool:
    d = ctypes.c_int32()
    _check(load().pg_server_poll(srv, ticket, ctypes.byref(d)))
    return bool(d.value)


def pg_server_wait(srv, ticket) -> float:
    lat = ctypes.c_double()
    _check(load().pg_server_wait(srv, ticket, ctypes.byref(lat)))
    return float(lat.value)


def pg_server_get_stats(srv) -> dict:
    st = _ServerStats()
    _check(load().pg_server_get_stats(srv, ctypes.byref(st)))
    return {f: int(getattr(st, f)) for f, _ in _ServerStats._fields_}


def pg_server_destroy(srv):
    _check(load().pg_server_destroy(srv))


# ---- handle classes ---------------------------------------------------------------

def _pairs(u, v):
    """Explicit pair lists as contiguous int32 tensors. (None, None) selects the
    graph's upper edges. An empty explicit list is returned as-is: callers must
    not pass it to the C ABI, where a NULL pointer (an empty tensor's data
    pointer) means "all upper edges"."""
    torch = _torch()
    if u is None and v is None:
        return None, None, 0
    if u is None or v is None:
        raise ValueError("give both u and v, or neither")
    if u.shape != v.shape:
        raise ValueError("u and v differ in length")
    return u.to(torch.int32).contiguous(), v.to(torch.int32).contiguous(), int(u.shape[0])


def _is_empty_explicit(u):
    return u is not None and u.shape[0] == 0


class Context:
    def __init__(self, device: int = 0):
        self.device = device
        self.h = pg_ctx_create(device)

    def close(self):
        if self.h:
            pg_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A device-resident CSR graph. ``offsets``/``adj`` may be numpy arrays
    (copied from the host) or int32 device tensors (copied, or borrowed)."""

    def __init__(self, ctx: Context, offsets, adj, validate: bool = False, borrow: bool = False, stream=None):
        torch = _torch()
        self.ctx = ctx
        flags = PG_VALIDATE if validate else 0
        if isinstance(offsets, np.ndarray):
            off = np.ascontiguousarray(offsets, dtype=np.int32)
            ad = np.ascontiguousarray(adj, dtype=np.int32)
            n, nnz = off.shape[0] - 1, ad.shape[0]
            self._keep = (off, ad)
            po = off.ctypes.data
            pa = ad.ctypes.data if nnz else None
        else:
            off = offsets.to(torch.int32).contiguous()
            ad = adj.to(torch.int32).contiguous()
            n, nnz = off.shape[0] - 1, ad.shape[0]
            flags |= PG_MEM_DEVICE | (PG_BORROW if borrow else 0)
            self._keep = (off, ad)
            po, pa = off.data_ptr(), (ad.data_ptr() if nnz else None)
        self.h = pg_graph_create(ctx.h, n, nnz, po, pa, flags, stream)
        info = pg_graph_get_info(self.h)
        self.n, self.nnz, self.m, self.max_degree = info.n, info.nnz, info.m, info.max_degree

    def close(self):
        if self.h:
            pg_graph_destroy(self.h)
            self.h = None

    def csr_fingerprint(self) -> str:
        """SHA-256 of the CSR arrays the graph was made from (offsets then adj, int32 little-endian)."""
        import hashlib
        off, ad = self._keep
        h = hashlib.sha256()
        for a in (off, ad):
            a = a if isinstance(a, np.ndarray) else a.cpu().numpy()
            h.update(np.ascontiguousarray(a, dtype="<i4").tobytes())
        return h.hexdigest()

    def upper_edges(self, stream=None):
        torch = _torch()
        dev = torch.device("cuda", self.ctx.device)
        eu = torch.empty(max(self.m, 1), dtype=torch.int32, device=dev)[: self.m]
        ev = torch.empty(max(self.m, 1), dtype=torch.int32, device=dev)[: self.m]
        if self.m:
            pg_graph_upper_edges(self.h, eu, ev, stream)
        return eu, ev

    def bits_for_budget(self, s: float) -> int:
        return pg_sketch_bits_for_budget(self.h, s)

    def build_sketches(self, kind, size: int, b: int = 1, seed: int = 1, oriented: bool = False,
                       stream=None) -> "Sketches":
        """Sketches of every N_v, or with oriented=True of the degree-oriented sets N+_v."""
        kind = KINDS.get(kind, kind) | (PG_ORIENTED if oriented else 0)
        return Sketches(self, pg_build_sketches(self.ctx.h, self.h, kind, size, b, seed, stream))

    def _dev(self):
        return _torch().device("cuda", self.ctx.device)

    def exact_intersect(self, u=None, v=None, algo=PG_EXACT_MERGE, stream=None):
        torch = _torch()
        u, v, npairs = _pairs(u, v)
        count = self.m if u is None else npairs
        out = torch.empty(max(count, 1), dtype=torch.int32, device=self._dev())[:count]
        if _is_empty_explicit(u):
            return out
        pg_exact_intersect_edges(self.ctx.h, self.h, algo, u, v, npairs, out if count else None, stream)
        return out

    def exact_tc(self, algo=PG_EXACT_MERGE, stream=None) -> int:
        return pg_exact_tc(self.ctx.h, self.h, algo, stream)

    def exact_cc(self, transitivity=False, stream=None):
        torch = _torch()
        cc = torch.empty(max(self.n, 1), dtype=torch.float32, device=self._dev())[: self.n]
        t = pg_exact_cc(self.ctx.h, self.h, cc, transitivity, stream)
        return (cc, t) if transitivity else cc

    def exact_jaccard(self, u=None, v=None, stream=None):
        torch = _torch()
        u, v, npairs = _pairs(u, v)
        count = self.m if u is None else npairs
        out = torch.empty(max(count, 1), dtype=torch.float32, device=self._dev())[:count]
        if _is_empty_explicit(u):
            return out
        pg_exact_jaccard(self.ctx.h, self.h, u, v, npairs, out, stream)
        return out

    def exact_similarity(self, measure, u=None, v=None, stream=None):
        """Exact similarity (``measure``: "cn", "jaccard", "overlap", "total" or a PG_SIM_* value), FP32."""
        torch = _torch()
        u, v, npairs = _pairs(u, v)
        count = self.m if u is None else npairs
        out = torch.empty(max(count, 1), dtype=torch.float32, device=self._dev())[:count]
        if _is_empty_explicit(u):
            return out
        pg_exact_similarity(self.ctx.h, self.h, SIMILARITIES.get(measure, measure), u, v, npairs,
                            out if count else None, stream)
        return out

    def exact_jarvis_patrick(self, measure, tau, algo=PG_EXACT_MERGE, stream=None):
        """(keep, kept): uint8 mask over the m upper edges of the exact clustering, and its size."""
        torch = _torch()
        keep = torch.empty(max(self.m, 1), dtype=torch.uint8, device=self._dev())[: self.m]
        kept = pg_exact_jarvis_patrick(self.ctx.h, self.h, algo, SIMILARITIES.get(measure, measure), tau,
                                       keep if self.m else None, True, stream)
        return keep, kept

    def import_sketches(self, kind, size: int, b: int, seed: int, rows, pc=None, oriented: bool = False,
                        stream=None) -> "Sketches":
        """A sketch set from exported rows (device uint8 [n, row_bytes]) without hashing."""
        kind = KINDS.get(kind, kind) | (PG_ORIENTED if oriented else 0)
        return Sketches(self, pg_sketches_import(self.ctx.h, self.h, kind, size, b, seed,
                                                 rows if self.n else None, pc if self.n else None, stream))

    def load_sketches(self, path, stream=None) -> "Sketches":
        """Resume a sketch set saved by Sketches.save (checks the graph's n, m and CSR fingerprint)."""
        import json
        torch = _torch()
        with np.load(path, allow_pickle=False) as f:
            header = json.loads(bytes(f["header"]).decode())
            rows = np.array(f["rows"])
            pc = np.array(f["pc"]) if "pc" in f.files else None
        if header.get("format") != SKETCH_FILE_FORMAT or header.get("hash_family") != HASH_FAMILY:
            raise ValueError(f"{path}: not a sketch file of this library's format and hash family")
        if header["n"] != self.n or header["m"] != self.m:
            raise ValueError(f"{path}: saved for a graph with n={header['n']} m={header['m']}, not n={self.n} m={self.m}")
        if header.get("csr_sha256") != self.csr_fingerprint():
            raise ValueError(f"{path}: saved for another graph of the same n and m (CSR fingerprints differ)")
        dev = self._dev()
        d_rows = torch.from_numpy(rows).to(dev)
        d_pc = torch.from_numpy(pc).to(dev) if pc is not None else None
        sk = self.import_sketches(header["kind"], header["size"], header["b"], header["seed"], d_rows, d_pc,
                                  oriented=header["oriented"], stream=stream)
        torch.cuda.synchronize(dev)
        return sk

    def exact_four_cliques(self, stream=None) -> int:
        """Exact 4-clique count (node iterator over oriented edges, Listing "lst:fcl")."""
        return pg_exact_four_cliques(self.ctx.h, self.h, stream)

    def clusters(self, keep=None, stream=None):
        """(labels, count): connected components of the kept upper edges (all edges if keep is None),
        each vertex labelled with the smallest vertex ID of its component."""
        torch = _torch()
        label = torch.empty(max(self.n, 1), dtype=torch.int32, device=self._dev())[: self.n]
        if keep is not None and keep.numel() != self.m:
            raise ValueError("keep must hold one byte per upper edge")
        count = pg_clusters(self.ctx.h, self.h, keep if (keep is not None and self.m) else None,
                            label if self.n else None, True, stream)
        return label, count


class Sketches:
    def __init__(self, graph: Graph, h):
        self.graph = graph
        self.h = h
        info = pg_sketches_get_info(h)
        self.oriented = bool(info.kind & PG_ORIENTED)
        self.kind, self.size, self.b, self.row_bytes = info.kind & ~PG_ORIENTED, info.size, info.b, info.row_bytes
        self.seed, self.total_bytes = info.seed, info.total_bytes

    def close(self):
        if self.h:
            pg_sketches_destroy(self.h)
            self.h = None

    def rebuild(self, seed=None, stream=None):
        """Recompute the rows in place (optionally from a new seed); allocates nothing."""
        seed = self.seed if seed is None else seed
        pg_sketches_rebuild(self.graph.ctx.h, self.h, seed, stream)
        self.seed = seed

    def export(self, stream=None):
        """(rows, pc): rows as uint8 [n, row_bytes] device tensor; pc int32 [n] or None."""
        torch = _torch()
        n = self.graph.n
        dev = self.graph._dev()
        rows = torch.empty((max(n, 1), self.row_bytes), dtype=torch.uint8, device=dev)[:n]
        pc = torch.empty(max(n, 1), dtype=torch.int32, device=dev)[:n] if self.kind == PG_BF else None
        if n:
            pg_sketches_export(self.h, rows, pc, stream)
        return rows, pc

    def intersect(self, estimator, u=None, v=None, want_est=True, want_raw=True, stream=None):
        torch = _torch()
        est_id = ESTIMATORS.get(estimator, estimator)
        u, v, npairs = _pairs(u, v)
        count = self.graph.m if u is None else npairs
        dev = self.graph._dev()
        est = torch.empty(max(count, 1), dtype=torch.float64, device=dev)[:count] if want_est else None
        raw = torch.empty(max(count, 1), dtype=torch.int32, device=dev)[:count] if want_raw else None
        if _is_empty_explicit(u):
            return est, raw
        pg_intersect_edges(self.graph.ctx.h, self.h, est_id, u, v, npairs, est if count else None,
                           raw if count else None, stream)
        return est, raw

    def tc(self, estimator, stream=None) -> float:
        return pg_tc(self.graph.ctx.h, self.h, ESTIMATORS.get(estimator, estimator), stream)

    def tc_async(self, estimator, out, stream=None):
        """Enqueue the estimate into out[0] (float64 device tensor) without waiting."""
        pg_tc_async(self.graph.ctx.h, self.h, ESTIMATORS.get(estimator, estimator), out, stream)
        return out

    def cc(self, estimator, transitivity=False, stream=None):
        torch = _torch()
        n = self.graph.n
        cc = torch.empty(max(n, 1), dtype=torch.float32, device=self.graph._dev())[:n]
        t = pg_cc(self.graph.ctx.h, self.h, ESTIMATORS.get(estimator, estimator), cc, transitivity, stream)
        return (cc, t) if transitivity else cc

    def jaccard(self, estimator, u=None, v=None, stream=None):
        torch = _torch()
        u, v, npairs = _pairs(u, v)
        count = self.graph.m if u is None else npairs
        out = torch.empty(max(count, 1), dtype=torch.float32, device=self.graph._dev())[:count]
        if _is_empty_explicit(u):
            return out
        pg_jaccard(self.graph.ctx.h, self.h, ESTIMATORS.get(estimator, estimator), u, v, npairs,
                   out if count else None, stream)
        return out

    def similarity(self, estimator, measure, u=None, v=None, stream=None):
        """Estimated similarity (``measure``: "cn", "jaccard", "overlap", "total" or a PG_SIM_* value), FP32."""
        torch = _torch()
        u, v, npairs = _pairs(u, v)
        count = self.graph.m if u is None else npairs
        out = torch.empty(max(count, 1), dtype=torch.float32, device=self.graph._dev())[:count]
        if _is_empty_explicit(u):
            return out
        pg_similarity(self.graph.ctx.h, self.h, ESTIMATORS.get(estimator, estimator),
                      SIMILARITIES.get(measure, measure), u, v, npairs, out if count else None, stream)
        return out

    def save(self, path, stream=None):
        """Checkpoint: the rows (and BF popcounts) with the parameters that rebuild them, as an .npz
        file (numeric arrays and a JSON header; loaded without pickle)."""
        import json
        rows, pc = self.export(stream)
        _torch().cuda.synchronize(rows.device)
        header = {"format": SKETCH_FILE_FORMAT, "hash_family": HASH_FAMILY, "kind": self.kind,
                  "oriented": self.oriented, "size": self.size, "b": self.b, "seed": self.seed,
                  "n": self.graph.n, "m": self.graph.m, "csr_sha256": self.graph.csr_fingerprint()}
        arrays = {"header": np.frombuffer(json.dumps(header).encode(), dtype=np.uint8),
                  "rows": rows.cpu().numpy()}
        if pc is not None:
            arrays["pc"] = pc.cpu().numpy()
        with open(path, "wb") as f:
            np.savez(f, **arrays)

    def four_cliques(self, stream=None) -> int:
        """4-clique estimate from Bloom filters of the oriented sets (build with oriented=True)."""
        return pg_four_cliques(self.graph.ctx.h, self.h, stream)

    def four_cliques_estimate(self, estimator="and", stream=None) -> float:
        """4-clique estimate with sketch intersections: |N+_w cap C3| from the filter of N+_w and a
        filter of C3 (estimators "and", "l", "pap" or "or"; Bloom filters of the oriented sets)."""
        return pg_four_cliques_estimate(self.graph.ctx.h, self.h, ESTIMATORS.get(estimator, estimator), stream)

    def jarvis_patrick(self, estimator, measure, tau, stream=None):
        """(keep, kept): uint8 mask over the m upper edges of the clustering (similarity > tau), and its size."""
        torch = _torch()
        m = self.graph.m
        keep = torch.empty(max(m, 1), dtype=torch.uint8, device=self.graph._dev())[:m]
        kept = pg_jarvis_patrick(self.graph.ctx.h, self.h, ESTIMATORS.get(estimator, estimator),
                                 SIMILARITIES.get(measure, measure), tau, keep if m else None, True, stream)
        return keep, kept


class Server:
    """Serving engine over resident sketch sets (see pg_server_* in probgraph.h).

    Requests are (op, sketch index, estimator, u, v) with host numpy int32
    arrays; results land in host numpy arrays (float64 for common neighbours,
    float32 for Jaccard)."""

    def __init__(self, graph: Graph, sketches, max_batches_in_flight=0, max_pairs_per_request=0,
                 max_batch_pairs=0, memory_budget_bytes=0):
        self.graph = graph
        self.sketches = list(sketches)
        p = _ServerParams(max_batches_in_flight, max_pairs_per_request, max_batch_pairs, memory_budget_bytes)
        self.h = pg_server_create(graph.ctx.h, graph.h, [sk.h for sk in self.sketches], p)
        self._keep = {}

    def make_request(self, op, sketch, estimator, u, v):
        u = np.ascontiguousarray(u, dtype=np.int32)
        v = np.ascontiguousarray(v, dtype=np.int32)
        # written once here, so that its pages are mapped before the server
        # first copies answers into it
        out = np.zeros(u.shape[0], dtype=np.float64 if op == PG_OP_CN else np.float32)
        out.fill(0)
        req = _Request(op, sketch, ESTIMATORS.get(estimator, estimator), 0, u.shape[0], u.ctypes.data,
                       v.ctypes.data, out.ctypes.data)
        return req, (u, v, out)

    def submit(self, op, sketch, estimator, u, v):
        """Returns (ticket, out array); raises PGError(PG_E_BUSY) when not admitted."""
        req, keep = self.make_request(op, sketch, estimator, u, v)
        t = pg_server_submit(self.h, req)
        self._keep[t] = keep
        return t, keep[2]

    def poll(self, ticket) -> bool:
        return pg_server_poll(self.h, ticket)

    def wait(self, ticket) -> float:
        lat = pg_server_wait(self.h, ticket)
        self._keep.pop(ticket, None)
        return lat

    def stats(self) -> dict:
        return pg_server_get_stats(self.h)

    def replay(self, requests, arrival_s=None, max_outstanding=0):
        """requests: list of (req struct, keep) from make_request. Returns
        (latency_ms array from arrival to result, elapsed seconds)."""
        n = len(requests)
        arr = (_Request * n)(*[r for r, _ in requests])
        lat = np.zeros(n, dtype=np.float64)
        el = ctypes.c_double()
        arrp = None
        if arrival_s is not None:
            arrival_s = np.ascontiguousarray(arrival_s, dtype=np.float64)
            arrp = arrival_s.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        _check(load().pg_server_replay(self.h, n, arr, arrp, max_outstanding,
                                       lat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(el)))
        return lat, float(el.value)

    def close(self):
        if self.h:
            pg_server_destroy(self.h)
            self.h = None


class Batch:
    """Many small graphs processed together (see pg_batch_* in probgraph.h).
    ``graphs``: objects with n, offsets, adj (numpy int32); ``bits``: per-graph
    Bloom-filter sizes."""

    def __init__(self, ctx: Context, graphs, bits, b: int = 1, seed: int = 1):
        lib = load()
        self.ctx = ctx
        self.count = len(graphs)
        self._keep = [(np.ascontiguousarray(g.offsets, np.int32), np.ascontiguousarray(g.adj, np.int32))
                      for g in graphs]
        offs = (_vp * self.count)(*[o.ctypes.data for o, _ in self._keep])
        adjs = (_vp * self.count)(*[a.ctypes.data if a.shape[0] else 0 for _, a in self._keep])
        ns = np.array([g.n for g in graphs], dtype=np.int32)
        nnz = np.array([a.shape[0] for _, a in self._keep], dtype=np.int64)
        bits = np.ascontiguousarray(bits, dtype=np.uint32)
        self.n_total = int(ns.sum())
        h = _vp()
        _check(lib.pg_batch_create(ctx.h, self.count, offs, adjs, ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   nnz.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   bits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), b, seed & (2**64 - 1),
                                   ctypes.byref(h)))
        self.h = h

    def set_params(self, tile_vertices=0, blocks_per_cu=0):
        _check(load().pg_batch_set_params(self.h, ctypes.byref(_BatchParams(tile_vertices, blocks_per_cu))))

    def params(self):
        p = _BatchParams()
        _check(load().pg_batch_get_params(self.h, ctypes.byref(p)))
        return int(p.tile_vertices), int(p.blocks_per_cu)

    def run(self, estimator="and", stream=None):
        _check(load().pg_batch_run(self.h, ESTIMATORS.get(estimator, estimator), _stream(stream)))

    def capture(self, estimator="and", stream=None):
        _check(load().pg_batch_capture(self.h, ESTIMATORS.get(estimator, estimator), _stream(stream)))

    def replay(self, stream=None):
        _check(load().pg_batch_replay(self.h, _stream(stream)))

    def results(self, stream=None):
        tc = np.zeros(self.count, dtype=np.float64)
        cc = np.zeros(max(self.n_total, 1), dtype=np.float32)
        _check(load().pg_batch_results(self.h, tc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       cc.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _stream(stream)))
        return tc, cc[: self.n_total]

    def autotune(self, estimator="and", stream=None):
        ms = ctypes.c_double()
        _check(load().pg_batch_autotune(self.h, ESTIMATORS.get(estimator, estimator), _stream(stream),
                                        ctypes.byref(ms)))
        return float(ms.value)

    def close(self):
        if self.h:
            _check(load().pg_batch_destroy(self.h))
            self.h = None
