// C ABI of the ProbGraph GPU library: argument checks, handle management and
// the sequencing of the device steps. Declarations and contracts live in
// include/probgraph.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "pg_device.h"
#include "pg_internal.h"

namespace pg {

namespace {
thread_local std::string g_last_error;
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
// Domain tags separating the hash constants of the three sketch kinds.
constexpr uint64_t kTagBF = 0x42462D48ull;  // "BF-H"
constexpr uint64_t kTagKH = 0x4B482D48ull;  // "KH-H"
constexpr uint64_t kTag1H = 0x31482D48ull;  // "1H-H"
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }
int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int dmalloc(void** p, size_t bytes, hipStream_t s) {
  *p = nullptr;
  if (bytes == 0) bytes = 8;
  const hipError_t e = hipMallocAsync(p, bytes, s);
  if (e == hipErrorOutOfMemory) return fail(PG_E_NOMEM, "device out of memory (" + std::to_string(bytes) + " bytes)");
  if (e != hipSuccess) return fail(PG_E_DEVICE, std::string("hipMallocAsync: ") + hipGetErrorString(e));
  return PG_OK;
}

int dfree(void* p, hipStream_t s) {
  if (!p) return PG_OK;
  PG_HIP(hipFreeAsync(p, s));
  return PG_OK;
}

int palloc(void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 8;
  const hipError_t e = hipMalloc(p, bytes);
  if (e == hipErrorOutOfMemory) return fail(PG_E_NOMEM, "device out of memory (" + std::to_string(bytes) + " bytes)");
  if (e != hipSuccess) return fail(PG_E_DEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
  return PG_OK;
}

int pfree(void* p) {
  if (!p) return PG_OK;
  PG_HIP(hipFree(p));
  return PG_OK;
}

// SplitMix64 used as a counter-based generator: output i of the stream whose
// initial state is `key` (Steele, Lea, Flood 2014).
uint64_t splitmix64(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * kGamma); }

// Hash constants of a sketch kind: a_i odd multipliers, c_i increments.
void hash_constants(int kind, uint64_t seed, uint32_t count, uint64_t* a, uint64_t* c) {
  const uint64_t key = seed ^ (kind == PG_BF ? kTagBF : kind == PG_MH_KHASH ? kTagKH : kTag1H);
  for (uint32_t i = 0; i < count; ++i) {
    a[i] = splitmix64(key, 2ull * i) | 1ull;
    c[i] = splitmix64(key, 2ull * i + 1);
  }
}

}  // namespace pg

using namespace pg;

namespace {

int use_device(const pg_ctx* ctx) {
  PG_HIP(hipSetDevice(ctx->device));
  return PG_OK;
}

void free_graph(pg_graph* g) {
  if (!g) return;
  free_graph(g->oriented);  // borrows poff/padj: freed before them
  if (g->owns_csr) {
    pfree(g->off);
    pfree(g->adj);
  }
  pfree(g->deg);
  pfree(g->eu);
  pfree(g->ev);
  pfree(g->arc_src);
  pfree(g->bin_verts);
  pfree(g->poff);
  pfree(g->padj);
  pfree(g->parc_src);
  pfree(g->ustart);
  pfree(g->upoff);
  free_plan(&g->plan_all);
  free_slabs(&g->slabs);
  free_slabs(&g->slabs_all);
  delete g;
}

void free_sketches(pg_sketches* sk) {
  if (!sk) return;
  pfree(sk->words);
  pfree(sk->pc);
  pfree(sk->sig);
  pfree(sk->ha);
  pfree(sk->hc);
  pfree(sk->table);
  pfree(sk->scratch);
  delete sk;
}

// Resolve a pair list: u = v = NULL selects the graph's upper edges.
int resolve_pairs(const pg_graph* g, const int32_t*& u, const int32_t*& v, int64_t& npairs) {
  if (!u && !v) {
    u = g->eu;
    v = g->ev;
    npairs = g->m;
    return PG_OK;
  }
  if (!u || !v) return fail(PG_E_INVALID, "u and v must both be given or both be NULL");
  if (npairs < 0) return fail(PG_E_INVALID, "npairs must be >= 0");
  return PG_OK;
}

// count (<= 8) 64-bit integers from the device into the context's pinned slot; waits.
int counts_to_host(pg_ctx* ctx, const unsigned long long* d, int count, hipStream_t s) {
  PG_HIP(hipMemcpyAsync(ctx->h_scalar, d, sizeof(unsigned long long) * (size_t)count, hipMemcpyDeviceToHost, s));
  PG_HIP(hipStreamSynchronize(s));
  return PG_OK;
}

int scalar_to_host(pg_ctx* ctx, const double* d_val, double* out, hipStream_t s) {
  PG_HIP(hipMemcpyAsync(ctx->h_scalar, d_val, sizeof(double), hipMemcpyDeviceToHost, s));
  PG_HIP(hipStreamSynchronize(s));
  *out = *ctx->h_scalar;
  return PG_OK;
}

}  // namespace

extern "C" {

const char* pg_last_error(void) { return g_last_error.c_str(); }

const char* pg_version(void) { return "probgraph-mi355x 0.1 (gfx950)"; }

int pg_ctx_create(int device, pg_ctx** out) {
  clear_error();
  if (!out) return fail(PG_E_INVALID, "out is NULL");
  *out = nullptr;
  int count = 0;
  PG_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(PG_E_INVALID, "device ordinal out of range");
  PG_HIP(hipSetDevice(device));
  pg_ctx* ctx = new (std::nothrow) pg_ctx();
  if (!ctx) return fail(PG_E_NOMEM, "host allocation failed");
  ctx->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->num_cus = prop.multiProcessorCount;
  // The library's per-call device temporaries (partial sums, workspaces)
  // come from the device's default stream-ordered pool. Its default release
  // threshold of 0 hands freed memory back at every synchronisation, so a
  // synchronous caller paid a fresh mapping per call (about 50 us for the
  // clustering coefficient's 4 MB of partial sums on R-MAT s20); keep up to
  // 1 GiB of freed memory in the pool for reuse.
  {
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess && pool) {
      uint64_t keep = 1ull << 30;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
  }
  if (hipHostMalloc((void**)&ctx->h_scalar, 64, hipHostMallocDefault) != hipSuccess) {
    delete ctx;
    return fail(PG_E_NOMEM, "pinned host allocation failed");
  }
  const int rc = noalloc_scratch(device, &ctx->scratch, &ctx->scratch_doubles);
  if (rc != PG_OK) {
    (void)hipHostFree(ctx->h_scalar);
    delete ctx;
    return rc;
  }
  *out = ctx;
  return PG_OK;
}

int pg_ctx_destroy(pg_ctx* ctx) {
  clear_error();
  if (!ctx) return fail(PG_E_INVALID, "ctx is NULL");
  if (ctx->h_scalar) (void)hipHostFree(ctx->h_scalar);
  delete ctx;
  return PG_OK;
}

int pg_graph_create(pg_ctx* ctx, int32_t n, int64_t nnz, const int32_t* offsets, const int32_t* adj, uint32_t flags,
                    void* stream, pg_graph** out) {
  clear_error();
  if (!ctx || !out) return fail(PG_E_INVALID, "ctx or out is NULL");
  *out = nullptr;
  if (n < 0) return fail(PG_E_INVALID, "n must be >= 0");
  if (nnz < 0 || nnz > (int64_t)INT32_MAX) return fail(PG_E_INVALID, "nnz must be in [0, 2^31 - 1]");
  if (!offsets || (nnz > 0 && !adj)) return fail(PG_E_INVALID, "offsets/adj is NULL");
  if ((flags & PG_BORROW) && !(flags & PG_MEM_DEVICE)) return fail(PG_E_INVALID, "PG_BORROW needs PG_MEM_DEVICE");
  if (flags & ~(PG_MEM_DEVICE | PG_BORROW | PG_VALIDATE)) return fail(PG_E_INVALID, "unknown flag bits");
  PG_TRY(use_device(ctx));
  hipStream_t s = (hipStream_t)stream;
  pg_graph* g = new (std::nothrow) pg_graph();
  if (!g) return fail(PG_E_NOMEM, "host allocation failed");
  g->ctx = ctx;
  g->n = n;
  g->nnz = nnz;
  int rc = PG_OK;
  const size_t off_bytes = sizeof(int32_t) * ((size_t)n + 1);
  const size_t adj_bytes = sizeof(int32_t) * (size_t)nnz;
  if ((flags & PG_MEM_DEVICE) && (flags & PG_BORROW)) {
    g->owns_csr = false;
    g->off = const_cast<int32_t*>(offsets);
    g->adj = const_cast<int32_t*>(adj);
  } else {
    g->owns_csr = true;
    const hipMemcpyKind kind = (flags & PG_MEM_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    rc = palloc((void**)&g->off, off_bytes);
    if (rc == PG_OK) rc = palloc((void**)&g->adj, adj_bytes);
    if (rc == PG_OK) {
      hipError_t e = hipMemcpyAsync(g->off, offsets, off_bytes, kind, s);
      if (e == hipSuccess && nnz > 0) e = hipMemcpyAsync(g->adj, adj, adj_bytes, kind, s);
      if (e != hipSuccess) rc = fail(PG_E_DEVICE, std::string("CSR copy: ") + hipGetErrorString(e));
    }
  }
  if (rc == PG_OK) rc = graph_prepare(g, (flags & PG_VALIDATE) != 0, s);
  if (rc == PG_OK) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = fail(PG_E_DEVICE, std::string("graph create: ") + hipGetErrorString(e));
  }
  if (rc != PG_OK) {
    (void)hipStreamSynchronize(s);
    free_graph(g);
    return rc;
  }
  *out = g;
  return PG_OK;
}

int pg_graph_destroy(pg_graph* g) {
  clear_error();
  if (!g) return fail(PG_E_INVALID, "graph is NULL");
  if (g->live_sketches > 0) return fail(PG_E_INVALID, "graph still has live sketches");
  PG_TRY(use_device(g->ctx));
  PG_HIP(hipDeviceSynchronize());
  free_graph(g);
  return PG_OK;
}

int pg_graph_get_info(const pg_graph* g, pg_graph_info* out) {
  clear_error();
  if (!g || !out) return fail(PG_E_INVALID, "NULL argument");
  out->n = g->n;
  out->max_degree = g->max_degree;
  out->nnz = g->nnz;
  out->m = g->m;
  return PG_OK;
}

int pg_graph_upper_edges(const pg_graph* g, int32_t* eu, int32_t* ev, void* stream) {
  clear_error();
  if (!g || !eu || !ev) return fail(PG_E_INVALID, "NULL argument");
  PG_TRY(use_device(g->ctx));
  if (g->m == 0) return PG_OK;
  hipStream_t s = (hipStream_t)stream;
  PG_HIP(hipMemcpyAsync(eu, g->eu, sizeof(int32_t) * g->m, hipMemcpyDeviceToDevice, s));
  PG_HIP(hipMemcpyAsync(ev, g->ev, sizeof(int32_t) * g->m, hipMemcpyDeviceToDevice, s));
  return PG_OK;
}

int pg_sketch_bits_for_budget(const pg_graph* g, double s, uint32_t* bits) {
  clear_error();
  if (!g || !bits) return fail(PG_E_INVALID, "NULL argument");
  if (!(s > 0.0 && s <= 1.0)) return fail(PG_E_INVALID, "budget must be in (0, 1]");
  if (g->n == 0) {
    *bits = 64;
    return PG_OK;
  }
  const double csr_bytes = 4.0 * ((double)g->n + 1.0) + 4.0 * (double)g->nnz;
  const double words = std::floor(s * 8.0 * csr_bytes / (64.0 * (double)g->n));
  const double b = std::max(64.0, 64.0 * words);
  *bits = (uint32_t)std::min(b, 4096.0);
  return PG_OK;
}

}  // extern "C"

namespace {

// A sketch set of the given parameters with its arrays allocated and hash
// constants in place; the rows are built (build = true) or left to the caller.
int make_sketches(pg_ctx* ctx, const pg_graph* gc, int kind, uint32_t size, uint32_t b, uint64_t seed,
                  hipStream_t s, bool build, pg_sketches** out) {
  if (!ctx || !gc || !out) return fail(PG_E_INVALID, "NULL argument");
  *out = nullptr;
  pg_graph* g = const_cast<pg_graph*>(gc);
  const bool oriented = (kind & PG_ORIENTED) != 0;
  kind &= ~PG_ORIENTED;
  if (kind == PG_BF) {
    if (size < 64 || size > 4096 || size % 64 != 0)
      return fail(PG_E_INVALID, "Bloom-filter size must be a multiple of 64 bits in [64, 4096]");
    if (b < 1 || b > 16) return fail(PG_E_INVALID, "b must be in [1, 16]");
  } else if (kind == PG_MH_KHASH || kind == PG_MH_1HASH) {
    if (size < 1 || size > 1024) return fail(PG_E_INVALID, "k must be in [1, 1024]");
    b = 1;
  } else {
    return fail(PG_E_INVALID, "unknown sketch kind");
  }
  PG_TRY(use_device(ctx));
  if (oriented) PG_TRY(graph_oriented(g, s));
  pg_graph* rows = oriented ? g->oriented : g;
  pg_sketches* sk = new (std::nothrow) pg_sketches();
  if (!sk) return fail(PG_E_NOMEM, "host allocation failed");
  sk->g = g;
  sk->rows = rows;
  sk->oriented = oriented;
  sk->kind = kind;
  sk->size = size;
  sk->b = b;
  sk->seed = seed;
  const size_t n = (size_t)std::max<int32_t>(g->n, 1);
  const uint32_t nh = kind == PG_BF ? b : (kind == PG_MH_KHASH ? size : 1);
  uint64_t ha[1024], hc[1024];
  hash_constants(kind, seed, nh, ha, hc);
  int rc = palloc((void**)&sk->ha, sizeof(uint64_t) * nh);
  if (rc == PG_OK) rc = palloc((void**)&sk->hc, sizeof(uint64_t) * nh);
  if (rc == PG_OK) {
    hipError_t e = hipMemcpyAsync(sk->ha, ha, sizeof(uint64_t) * nh, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(sk->hc, hc, sizeof(uint64_t) * nh, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host arrays are on this stack frame
    if (e != hipSuccess) rc = fail(PG_E_DEVICE, std::string("hash constants: ") + hipGetErrorString(e));
  }
  if (kind == PG_BF) {
    sk->W = size / 64;
    if (rc == PG_OK) rc = palloc((void**)&sk->words, sizeof(uint64_t) * (bf_total_words((int64_t)n, sk->W) + kBfSlackWords));
    if (rc == PG_OK) rc = palloc((void**)&sk->pc, sizeof(uint32_t) * n);
    if (rc == PG_OK) rc = palloc((void**)&sk->table, sizeof(double) * kBfTables * (size + 1));
    if (rc == PG_OK) rc = fill_tables(sk, s);
    if (rc == PG_OK)
      rc = palloc((void**)&sk->scratch, sizeof(uint64_t) * sk->W * (size_t)std::max<int64_t>(rows->plan_all.n_chunks, 1));
    if (rc == PG_OK && build && g->n > 0) rc = build_bf(sk, s);
  } else {
    if (rc == PG_OK) rc = palloc((void**)&sk->sig, sizeof(uint32_t) * size * n);
    if (rc == PG_OK && kind == PG_MH_KHASH) {  // chunk partials of heavy vertices: k keys and k elements per chunk
      const size_t slots = (size_t)size * (size_t)std::max<int64_t>(rows->plan_all.n_chunks, 1);
      rc = palloc((void**)&sk->scratch, sizeof(uint64_t) * (slots + (slots + 1) / 2));
    }
    if (rc == PG_OK && kind == PG_MH_1HASH && size <= (uint32_t)kHeavyChunk && rows->plan_all.n_chunks > 0) {
      // heavy vertices' chunk candidates: k elements per chunk
      const size_t slots = (size_t)size * (size_t)rows->plan_all.n_chunks;
      rc = palloc((void**)&sk->scratch, sizeof(uint64_t) * ((slots + 1) / 2));
    }
    if (rc == PG_OK && build && g->n > 0) rc = kind == PG_MH_KHASH ? build_khash(sk, s) : build_onehash(sk, s);
  }
  if (rc != PG_OK) {
    (void)hipStreamSynchronize(s);
    free_sketches(sk);
    return rc;
  }
  *out = sk;
  return PG_OK;
}

}  // namespace

extern "C" {

int pg_build_sketches(pg_ctx* ctx, const pg_graph* gc, int kind, uint32_t size, uint32_t b, uint64_t seed,
                      void* stream, pg_sketches** out) {
  clear_error();
  pg_sketches* sk = nullptr;
  PG_TRY(make_sketches(ctx, gc, kind, size, b, seed, (hipStream_t)stream, true, &sk));
  sk->g->live_sketches++;
  *out = sk;
  return PG_OK;
}

int pg_sketches_import(pg_ctx* ctx, const pg_graph* gc, int kind, uint32_t size, uint32_t b, uint64_t seed,
                       const void* rows, const uint32_t* pc, void* stream, pg_sketches** out) {
  clear_error();
  if (gc && gc->n > 0 && !rows) return fail(PG_E_INVALID, "rows is NULL");
  hipStream_t s = (hipStream_t)stream;
  pg_sketches* sk = nullptr;
  PG_TRY(make_sketches(ctx, gc, kind, size, b, seed, s, false, &sk));
  const size_t n = (size_t)sk->g->n;
  int rc = PG_OK;
  if (n > 0) {
    if (sk->kind == PG_BF) {
      rc = bf_pack(sk, rows, pc, s);
    } else if (hipMemcpyAsync(sk->sig, rows, n * sk->size * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) {
      rc = fail(PG_E_DEVICE, "row copy failed");
    }
  }
  if (rc != PG_OK) {
    (void)hipStreamSynchronize(s);
    free_sketches(sk);
    return rc;
  }
  sk->g->live_sketches++;
  *out = sk;
  return PG_OK;
}

int pg_sketches_rebuild(pg_ctx* ctx, pg_sketches* sk, uint64_t seed, void* stream) {
  clear_error();
  if (!ctx || !sk) return fail(PG_E_INVALID, "NULL argument");
  PG_TRY(use_device(ctx));
  hipStream_t s = (hipStream_t)stream;
  if (seed != sk->seed) {
    const uint32_t nh = sk->kind == PG_BF ? sk->b : (sk->kind == PG_MH_KHASH ? sk->size : 1);
    uint64_t ha[1024], hc[1024];
    hash_constants(sk->kind, seed, nh, ha, hc);
    PG_HIP(hipMemcpyAsync(sk->ha, ha, sizeof(uint64_t) * nh, hipMemcpyHostToDevice, s));
    PG_HIP(hipMemcpyAsync(sk->hc, hc, sizeof(uint64_t) * nh, hipMemcpyHostToDevice, s));
    PG_HIP(hipStreamSynchronize(s));  // the host arrays are on this stack frame
    sk->seed = seed;
  }
  if (sk->g->n == 0) return PG_OK;
  if (sk->kind == PG_BF) return build_bf(sk, s);
  if (sk->kind == PG_MH_KHASH) return build_khash(sk, s);
  return build_onehash(sk, s);
}

int pg_sketches_destroy(pg_sketches* sk) {
  clear_error();
  if (!sk) return fail(PG_E_INVALID, "sketches is NULL");
  PG_TRY(use_device(sk->g->ctx));
  PG_HIP(hipDeviceSynchronize());
  sk->g->live_sketches--;
  free_sketches(sk);
  return PG_OK;
}

int pg_sketches_get_info(const pg_sketches* sk, pg_sketch_info* out) {
  clear_error();
  if (!sk || !out) return fail(PG_E_INVALID, "NULL argument");
  out->kind = sk->kind | (sk->oriented ? PG_ORIENTED : 0);
  out->size = sk->size;
  out->b = sk->b;
  out->seed = sk->seed;
  out->row_bytes = sk->kind == PG_BF ? sk->size / 8 : sk->size * 4;
  out->total_bytes = (uint64_t)out->row_bytes * (uint64_t)sk->g->n + (sk->kind == PG_BF ? 4ull * sk->g->n : 0ull);
  return PG_OK;
}

int pg_sketches_export(const pg_sketches* sk, void* rows, uint32_t* pc, void* stream) {
  clear_error();
  if (!sk) return fail(PG_E_INVALID, "sketches is NULL");
  PG_TRY(use_device(sk->g->ctx));
  hipStream_t s = (hipStream_t)stream;
  const size_t n = (size_t)sk->g->n;
  if (n == 0) return PG_OK;
  if (rows) {
    if (sk->kind == PG_BF)
      PG_TRY(bf_unpack(sk, rows, s));
    else
      PG_HIP(hipMemcpyAsync(rows, sk->sig, n * sk->size * 4, hipMemcpyDeviceToDevice, s));
  }
  if (pc) {
    if (sk->kind != PG_BF) return fail(PG_E_INVALID, "popcounts exist only for Bloom filters");
    PG_HIP(hipMemcpyAsync(pc, sk->pc, n * 4, hipMemcpyDeviceToDevice, s));
  }
  return PG_OK;
}

int pg_intersect_edges(pg_ctx* ctx, const pg_sketches* sk, int estimator, const int32_t* u, const int32_t* v,
                       int64_t npairs, double* est, uint32_t* raw, void* stream) {
  clear_error();
  if (!ctx || !sk) return fail(PG_E_INVALID, "NULL argument");
  PG_TRY(resolve_pairs(sk->g, u, v, npairs));
  PG_TRY(use_device(ctx));
  return estimate_pairs(sk, estimator, u, v, npairs, est, raw, nullptr, PG_SIM_COMMON, (hipStream_t)stream);
}

int pg_tc(pg_ctx* ctx, const pg_sketches* sk, int estimator, double* tc, void* stream) {
  clear_error();
  if (!ctx || !sk || !tc) return fail(PG_E_INVALID, "NULL argument");
  PG_TRY(use_device(ctx));
  hipStream_t s = (hipStream_t)stream;
  double* d = nullptr;
  PG_TRY(dmalloc((void**)&d, sizeof(double), s));
  int rc = estimate_tc(sk, estimator, d, s);
  if (rc == PG_OK) rc = scalar_to_host(ctx, d, tc, s);
  dfree(d, s);
  return rc;
}

int pg_tc_async(pg_ctx* ctx, const pg_sketches* sk, int estimator, double* d_tc, void* stream) {
  clear_error();
  if (!ctx || !sk || !d_tc) return fail(PG_E_INVALID, "NULL argument");
  PG_TRY(use_device(ctx));
  return estimate_tc(sk, estimator, d_tc, (hipStream_t)stream);
}

int pg_tc_noalloc(pg_ctx* ctx, const pg_sketches* sk, int estimator, double* d_tc, void* stream) {
  clear_error();
  if (!ctx || !sk || !d_tc) return fail(PG_E_INVALID, "NULL argument");
  if (!ctx->scratch) return fail(PG_E_DEVICE, "the context has no fixed workspace");
  PG_TRY(use_device(ctx));
  const TcWorkspace ws{ctx->scratch, ctx->scratch_doubles};
  return estimate_tc(sk, estimator, d_tc, (hipStream_t)stream, &ws);
}

int pg_cc(pg_ctx* ctx, const pg_sketches* sk, int estimator, float* cc, double* transitivity, void* stream) {
  clear_error();
  if (!ctx || !sk || !cc) return fail(PG_E_INVALID, "NULL argument");
  PG_TRY(use_device(ctx));
  hipStream_t s = (hipStream_t)stream;
  const pg_graph* g = sk->g;
  double* vsum = nullptr;
  if (transitivity) PG_TRY(dmalloc((void**)&vsum, sizeof(double) * ((size_t)g->n + 1), s));
  int rc = estimate_cc(sk, estimator, cc, vsum, s);
  if (rc == PG_OK && transitivity) {
    // sum_v sum_{u in N_v} I^ counts every edge twice: 3 TC^ = (1/2) sum_v S_v
    rc = sum_array(vsum, g->n, 2.0, vsum + g->n, s);
    double three_tc = 0.0;
    if (rc == PG_OK) rc = scalar_to_host(ctx, vsum + g->n, &three_tc, s);
    if (rc == PG_OK) *transitivity = g->wedges ? three_tc / (double)g->wedges : 0.0;
  }
  if (vsum) dfree(vsum, s);
  return rc;
}

int pg_jaccard(pg_ctx* ctx, const pg_sketches* sk, int estimator, const int32_t* u, const int32_t* v, int64_t npairs,
               float* out, void* stream) {
  clear_error();
  if (!ctx || !sk) return fail(PG_E_INVALID, "NULL argument");
  PG_TRY(resolve_pairs(sk->g, u, v, npairs));
  if (npairs > 0 && !out) return fail(PG_E_INVALID, "out is NULL");
  PG_TRY(use_device(ctx));
  return estimate_pairs(sk, estimator, u, v, npairs, nullptr, nullptr, out, PG_SIM_JACCARD, (hipStream_t)stream);
}

int pg_similarity(pg_ctx* ctx, const pg_sketches* sk, int estimator, int measure, const int32_t* u, const int32_t* v,
                  int64_t npairs, float* out, void* stream) {
  clear_error();
  if (!ctx || !sk) return fail(PG_E_INVALID, "NULL argument");
  if (measure < PG_SIM_COMMON || measure > PG_SIM_TOTAL) return fail(PG_E_INVALID, "unknown similarity measure");
  PG_TRY(resolve_pairs(sk->g, u, v, npairs));
  if (npairs > 0 && !out) return fail(PG_E_INVALID, "out is NULL");
  PG_TRY(use_device(ctx));
  return estimate_pairs(sk, estimator, u, v, npairs, nullptr, nullptr, out, measure, (hipStream_t)stream);
}

int pg_jarvis_patrick(pg_ctx* ctx, const pg_sketches* sk, int estimator, int measure, double tau, uint8_t* keep,
                      int64_t* kept, void* stream) {
  clear_error();
  if (!ctx || !sk) return fail(PG_E_INVALID, "NULL argument");
  if (!keep && !kept) return fail(PG_E_INVALID, "keep and kept are both NULL");
  if (std::isnan(tau)) return fail(PG_E_INVALID, "tau is NaN");
  PG_TRY(use_device(ctx));
  hipStream_t s = (hipStream_t)stream;
  unsigned long long* d = nullptr;
  PG_TRY(dmalloc((void**)&d, sizeof(unsigned long long), s));
  int rc = estimate_jp(sk, estimator, measure, tau, keep, d, s);
  if (rc == PG_OK && kept) rc = counts_to_host(ctx, d, 1, s);
  if (rc == PG_OK && kept) *kept = (int64_t)((const unsigned long long*)ctx->h_scalar)[0];
  dfree(d, s);
  return rc;
}

int pg_exact_intersect_edges(pg_ctx* ctx, const pg_graph* g, int algo, const int32_t* u, const int32_t* v,
                             int64_t npairs, uint32_t* out, void* stream) {
  clear_error();
  if (!ctx || !g) return fail(PG_E_INVALID, "NULL argument");
  PG_TRY(resolve_pairs(g, u, v, npairs));
  if (npairs > 0 && !out) return fail(PG_E_INVALID, "out is NULL");
  PG_TRY(use_device(ctx));
  return exact_pairs(g, algo, u, v, npairs, out, (hipStream_t)stream);
}

int pg_exact_tc(pg_ctx* ctx, const pg_graph* gc, int algo, uint64_t* tc, void* stream) {
  clear_error();
  if (!ctx || !gc || !tc) return fail(PG_E_INVALID, "NULL argument");
  PG_TRY(use_device(ctx));
  hipStream_t s = (hipStream_t)stream;
  uint64_t* d = nullptr;
  PG_TRY(dmalloc((void**)&d, sizeof(uint64_t), s));
  int rc = exact_tc(const_cast<pg_graph*>(gc), algo, d, s);
  if (rc == PG_OK) {
    hipError_t e = hipMemcpyAsync(ctx->h_scalar, d, sizeof(uint64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess)
      rc = fail(PG_E_DEVICE, std::string("exact tc: ") + hipGetErrorString(e));
    else
      std::memcpy(tc, ctx->h_scalar, sizeof(uint64_t));
  }
  dfree(d, s);
  return rc;
}

int pg_exact_cc(pg_ctx* ctx, const pg_graph* gc, float* cc, double* transitivity, void* stream) {
  clear_error();
  if (!ctx || !gc || !cc) return fail(PG_E_INVALID, "NULL argument");
  PG_TRY(use_device(ctx));
  pg_graph* g = const_cast<pg_graph*>(gc);
  PG_TRY(exact_cc(g, cc, (hipStream_t)stream));
  if (transitivity) {
    uint64_t tc = 0;
    PG_TRY(pg_exact_tc(ctx, g, PG_EXACT_MERGE, &tc, stream));
    *transitivity = g->wedges ? 3.0 * (double)tc / (double)g->wedges : 0.0;
  }
  return PG_OK;
}

int pg_exact_jaccard(pg_ctx* ctx, const pg_graph* g, const int32_t* u, const int32_t* v, int64_t npairs, float* out,
                     void* stream) {
  return pg_exact_similarity(ctx, g, PG_SIM_JACCARD, u, v, npairs, out, stream);
}

int pg_exact_similarity(pg_ctx* ctx, const pg_graph* g, int measure, const int32_t* u, const int32_t* v,
                        int64_t npairs, float* out, void* stream) {
  clear_error();
  if (!ctx || !g) return fail(PG_E_INVALID, "NULL argument");
  if (measure < PG_SIM_COMMON || measure > PG_SIM_TOTAL) return fail(PG_E_INVALID, "unknown similarity measure");
  PG_TRY(resolve_pairs(g, u, v, npairs));
  if (npairs > 0 && !out) return fail(PG_E_INVALID, "out is NULL");
  PG_TRY(use_device(ctx));
  return exact_similarity(g, measure, u, v, npairs, out, (hipStream_t)stream);
}

int pg_exact_jarvis_patrick(pg_ctx* ctx, const pg_graph* g, int algo, int measure, double tau, uint8_t* keep,
                            int64_t* kept, void* stream) {
  clear_error();
  if (!ctx || !g) return fail(PG_E_INVALID, "NULL argument");
  if (!keep && !kept) return fail(PG_E_INVALID, "keep and kept are both NULL");
  if (std::isnan(tau)) return fail(PG_E_INVALID, "tau is NaN");
  PG_TRY(use_device(ctx));
  hipStream_t s = (hipStream_t)stream;
  unsigned long long* d = nullptr;
  PG_TRY(dmalloc((void**)&d, sizeof(unsigned long long), s));
  int rc = exact_jp(g, algo, measure, tau, keep, d, s);
  if (rc == PG_OK && kept) rc = counts_to_host(ctx, d, 1, s);
  if (rc == PG_OK && kept) *kept = (int64_t)((const unsigned long long*)ctx->h_scalar)[0];
  dfree(d, s);
  return rc;
}

int pg_exact_four_cliques(pg_ctx* ctx, const pg_graph* gc, uint64_t* count, void* stream) {
  clear_error();
  if (!ctx || !gc || !count) return fail(PG_E_INVALID, "NULL argument");
  PG_TRY(use_device(ctx));
  hipStream_t s = (hipStream_t)stream;
  unsigned long long* d = nullptr;
  PG_TRY(dmalloc((void**)&d, sizeof(unsigned long long), s));
  int rc = four_cliques(const_cast<pg_graph*>(gc), nullptr, d, s);
  if (rc == PG_OK) rc = counts_to_host(ctx, d, 1, s);
  if (rc == PG_OK) *count = (uint64_t)((const unsigned long long*)ctx->h_scalar)[0];
  dfree(d, s);
  return rc;
}

int pg_four_cliques(pg_ctx* ctx, const pg_sketches* sk, uint64_t* count, void* stream) {
  clear_error();
  if (!ctx || !sk || !count) return fail(PG_E_INVALID, "NULL argument");
  if (sk->kind != PG_BF || !sk->oriented)
    return fail(PG_E_INVALID, "4-cliques need Bloom filters of the oriented sets (PG_BF | PG_ORIENTED)");
  PG_TRY(use_device(ctx));
  hipStream_t s = (hipStream_t)stream;
  unsigned long long* d = nullptr;
  PG_TRY(dmalloc((void**)&d, sizeof(unsigned long long), s));
  int rc = four_cliques(sk->g, sk, d, s);
  if (rc == PG_OK) rc = counts_to_host(ctx, d, 1, s);
  if (rc == PG_OK) *count = (uint64_t)((const unsigned long long*)ctx->h_scalar)[0];
  dfree(d, s);
  return rc;
}

int pg_four_cliques_estimate(pg_ctx* ctx, const pg_sketches* sk, int estimator, double* count, void* stream) {
  clear_error();
  if (!ctx || !sk || !count) return fail(PG_E_INVALID, "NULL argument");
  if (sk->kind != PG_BF || !sk->oriented)
    return fail(PG_E_INVALID, "4-cliques need Bloom filters of the oriented sets (PG_BF | PG_ORIENTED)");
  PG_TRY(use_device(ctx));
  hipStream_t s = (hipStream_t)stream;
  double* d = nullptr;
  PG_TRY(dmalloc((void**)&d, sizeof(double), s));
  int rc = four_cliques_estimate(sk, estimator, d, s);
  if (rc == PG_OK) rc = scalar_to_host(ctx, d, count, s);
  dfree(d, s);
  return rc;
}

int pg_clusters(pg_ctx* ctx, const pg_graph* g, const uint8_t* keep, int32_t* label, int64_t* nclusters,
                void* stream) {
  clear_error();
  if (!ctx || !g) return fail(PG_E_INVALID, "NULL argument");
  if (g->n > 0 && !label) return fail(PG_E_INVALID, "label is NULL");
  PG_TRY(use_device(ctx));
  hipStream_t s = (hipStream_t)stream;
  unsigned long long* d = nullptr;
  PG_TRY(dmalloc((void**)&d, 2 * sizeof(unsigned long long), s));
  int rc = clusters(g, keep, label, d, s);
  if (rc == PG_OK && nclusters) {
    rc = counts_to_host(ctx, d, 2, s);
    const unsigned long long* h = (const unsigned long long*)ctx->h_scalar;
    if (rc == PG_OK && h[1]) rc = fail(PG_E_DEVICE, "cluster union did not settle");
    if (rc == PG_OK) *nclusters = (int64_t)h[0];
  }
  dfree(d, s);
  return rc;
}

}  // extern "C"
