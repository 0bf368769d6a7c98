// Intersection estimates over vertex pairs (Sections 4.2-4.4) and the
// quantities built from them: the triangle-count sum (Section 7), local
// clustering coefficients, vertex similarities (Listing "lst:sim") and
// Jarvis-Patrick clustering (Listing "lst:cl").
//
// Every pair is independent: one lane per pair gathers the two sketch rows,
// reduces them to an integer count (ones of the AND or OR of two filters,
// positional matches of two k-hash rows, or the bottom-k union walk of two
// 1-hash rows) and maps the count to an FP64 estimate. Sums use a fixed
// chunking of the pair list and a fixed reduction tree, so they are
// bit-reproducible and independent of the launch configuration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <type_traits>

#include "pg_device.h"
#include "pg_internal.h"
#include "pg_pair.h"

// ---- fixed workspace of pg_tc_noalloc -------------------------------------------
// Partial sums of the triangle count for callers that cannot allocate device
// memory. Every GPU the library runs on holds its own copy of this array until
// the process ends. In host code the name stands for a host-side shadow, not a
// device address: host code uses only the address hipGetSymbolAddress returns
// on each device (noalloc_scratch below).
constexpr int64_t kScratchDoubles = (int64_t)1 << 21;  // 16 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace pg {
namespace {

constexpr int kBlock = 256;
constexpr int kChunkItems = 8;
constexpr int64_t kChunk = (int64_t)kBlock * kChunkItems;  // pairs per chunk partial
constexpr int kCountBlocksPerCu = 8;  // grid of kernels that count into one global counter
// The vertex-centric 1-hash kernels count matches of the union walk (union
// and literal readings); the KMV estimators take the general per-pair path.
inline bool is_minhash_ratio(int est) { return est == PG_EST_MH_1HASH || est == PG_EST_MH_1HASH_LITERAL; }
// Estimators of 1-hash rows that the vertex-centric union counts serve.
inline bool is_onehash_union(int est) {
  return is_minhash_ratio(est) || est == PG_EST_KMV || est == PG_EST_KMV_SKETCH_SIZES;
}

constexpr const char* kOrientedNeedsNv =
    "defined on N_v: an oriented sketch set (PG_ORIENTED) serves intersections and the triangle count";

// ---- kernels -------------------------------------------------------------------

template <int KIND, int WT>
__global__ __launch_bounds__(kBlock) void k_pairs(SkView s, const int32_t* __restrict__ pu,
                                                  const int32_t* __restrict__ pv, int64_t npairs,
                                                  double* __restrict__ est_out, uint32_t* __restrict__ raw_out,
                                                  float* __restrict__ sim_out, int measure) {
  for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < npairs; e += (int64_t)gridDim.x * kBlock) {
    const int32_t u = pu[e], v = pv[e];
    uint32_t raw;
    const double est = eval_pair<KIND, WT>(s, u, v, raw);
    if (est_out) est_out[e] = est;
    if (raw_out) raw_out[e] = raw;
    if (sim_out) {
      const bool ok = (uint32_t)u < (uint32_t)s.n && (uint32_t)v < (uint32_t)s.n;
      sim_out[e] = ok ? (float)similarity_of(measure, est, s.deg[u], s.deg[v]) : __int_as_float(0x7FC00000);
    }
  }
}

// Jarvis-Patrick selection over the m upper edges: keep[e] = (similarity > tau)
// in FP64, and |C| added to *kept once per block (integer atomics, so the
// count does not depend on scheduling).
template <int KIND, int WT>
__global__ __launch_bounds__(kBlock) void k_pairs_jp(SkView s, const int32_t* __restrict__ pu,
                                                     const int32_t* __restrict__ pv, int64_t npairs, int measure,
                                                     double tau, uint8_t* __restrict__ keep,
                                                     unsigned long long* __restrict__ kept) {
  __shared__ uint32_t block_kept;
  if (threadIdx.x == 0) block_kept = 0;
  __syncthreads();
  uint32_t mine = 0;
  for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < npairs; e += (int64_t)gridDim.x * kBlock) {
    const int32_t u = pu[e], v = pv[e];
    uint32_t raw;
    const double est = eval_pair<KIND, WT>(s, u, v, raw);
    const bool in = similarity_of(measure, est, s.deg[u], s.deg[v]) > tau;
    if (keep) keep[e] = in ? 1 : 0;
    mine += in ? 1u : 0u;
  }
  if (mine) atomicAdd(&block_kept, mine);
  __syncthreads();
  if (threadIdx.x == 0 && block_kept) atomicAdd(kept, (unsigned long long)block_kept);
}

// Partial sums over fixed chunks of kChunk pairs: thread t of the chunk adds
// pairs chunk*kChunk + j*kBlock + t, j = 0..7, then a fixed tree.
template <int KIND, int WT>
__global__ __launch_bounds__(kBlock) void k_pairs_sum(SkView s, const int32_t* __restrict__ pu,
                                                      const int32_t* __restrict__ pv, int64_t npairs,
                                                      double* __restrict__ chunks) {
  __shared__ double lds[kBlock / kWave];
  const int64_t nchunks = (npairs + kChunk - 1) / kChunk;
  for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < kChunkItems; ++j) {
      const int64_t e = ch * kChunk + (int64_t)j * kBlock + threadIdx.x;
      if (e < npairs) {
        uint32_t raw;
        acc += eval_pair<KIND, WT>(s, pu[e], pv[e], raw);
      }
    }
    const double r = block_sum_256(acc, lds);
    if (threadIdx.x == 0) chunks[ch] = r;
  }
}

// cc_v = sum_{u in N_v} I^(u, v) / (d_v (d_v - 1)); G lanes per vertex, fixed order.
template <int KIND, int WT, int G>
__global__ __launch_bounds__(kBlock) void k_cc(SkView s, const int32_t* __restrict__ off,
                                               const int32_t* __restrict__ adj, const int32_t* __restrict__ verts,
                                               int64_t nverts, float* __restrict__ cc, double* __restrict__ vsum) {
  __shared__ double lds[kBlock / kWave];
  const int64_t grp = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x % G;
  const bool active = grp < nverts;
  const int32_t v = active ? verts[grp] : 0;
  double acc = 0.0;
  if (active) {
    for (int64_t p = off[v] + lane; p < off[v + 1]; p += G) {
      uint32_t raw;
      acc += eval_pair<KIND, WT>(s, v, adj[p], raw);
    }
  }
  double tot;
  if constexpr (G <= kWave) {
    tot = group_sum<G>(acc);
  } else {
    tot = block_sum_256(acc, lds);
  }
  if (active && lane == 0) {
    const int32_t d = s.deg[v];
    const double val = d >= 2 ? tot / ((double)d * ((double)d - 1.0)) : 0.0;
    cc[v] = (float)val;
    if (vsum) vsum[v] = tot;
  }
}

// ---- triangle count over the upper-neighbour plan (Bloom filters, W <= 16) ----
//
// Vertex-centric: the group owning v keeps B_v in registers and walks the
// neighbours above v straight from the CSR, gathering U rows ahead before
// reducing any of them. A neighbour row is read by a team of T lanes side by
// side, lane k holding words [kQ, kQ + Q) of B_v and loading the same words of
// the row (Q = ceil(W / T), 16-byte loads); the team's counts meet in quad DPP
// adds. Scattered row reads are limited by the L1 address and data path, not
// by bytes: two lanes per row cut the cache accesses per row, while wider
// teams cost more VALU work than they save (measured on gfx950). The last
// lane of a team may read up to Q-1 words past the row (the next row, the
// group padding, or the slack words after the last group); the matching words
// of B_v are zero, so they never count. The estimator table sits in LDS.
// Every block writes one partial sum; the final fixed-order sum makes the
// result independent of scheduling.

template <int W>
struct RowUnroll {
  static constexpr int value = W <= 4 ? 8 : (W <= 8 ? 4 : 2);
};

constexpr int kTcTeamMax = 2;  // lanes per row at most (within a quad, so DPP can reduce)

// Lanes per row for a group of G lanes: enough 16-byte loads to cover W
// words, at most kTcTeamMax and at most G.
template <int W, int G>
struct TcTeam {
  static constexpr int want = W <= 2 ? 1 : (W <= 4 ? 2 : 4);
  static constexpr int capped = want < kTcTeamMax ? want : kTcTeamMax;
  static constexpr int value = capped < G ? capped : G;
  static constexpr int words = (W + value - 1) / value;  // Q
};

// Words [kQ, kQ + Q) of row v for team member k, zero past the row's end.
template <int W, int G>
__device__ __forceinline__ void load_team_row(const uint64_t* __restrict__ words, int32_t v, int k,
                                              uint64_t (&r)[TcTeam<W, G>::words]) {
  constexpr int Q = TcTeam<W, G>::words;
  const uint64_t* p = words + bf_row_offset(v, W) + k * Q;
#pragma unroll
  for (int i = 0; i < Q; ++i) r[i] = (k * Q + i < W) ? p[i] : 0;
}

template <int W, int U, int G, bool OR>
__device__ __forceinline__ double bf_row_sum(const SkView& s, const uint64_t (&ru)[TcTeam<W, G>::words], int32_t du,
                                             uint32_t pcu, const int32_t* __restrict__ adj, int64_t beg, int64_t end,
                                             int lane, const double* __restrict__ tab) {
  constexpr int T = TcTeam<W, G>::value;
  constexpr int Q = TcTeam<W, G>::words;
  constexpr int NT = G / T;  // teams in the group
  static_assert(G % T == 0, "a group holds whole teams");
  const int k = lane % T;
  const bool reads = k * Q < W;  // members past the row's end load nothing
  double acc = 0.0;
  // every member of a team takes the same trip count, so the DPP adds only
  // read lanes that are active
  for (int64_t p0 = beg + lane / T; p0 < end; p0 += (int64_t)NT * U) {
    int32_t x[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int64_t p = p0 + (int64_t)j * NT;
      x[j] = p < end ? adj[p] : -1;
    }
    uint64_t rv[U][Q];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      if (x[j] >= 0 && reads) {
        const uint64_t* r = s.words + bf_row_offset(x[j], W) + k * Q;
#pragma unroll
        for (int i = 0; i < Q; ++i) rv[j][i] = r[i];
      } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) rv[j][i] = 0;
      }
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      uint32_t c = 0;
#pragma unroll
      for (int i = 0; i < Q; ++i) c += (uint32_t)__popcll(ru[i] & rv[j][i]);
      c = team_sum<T>(c);
      if (k == 0 && x[j] >= 0) {
        if constexpr (OR)
          acc += ((double)du + (double)s.deg[x[j]]) + tab[pcu + s.pc[x[j]] - c];
        else
          acc += tab[c];
      }
    }
  }
  return acc;
}

// Per-edge outputs of one group's upper neighbours adj[beg, end) of v (the
// pair kernel's values, bit for bit): edge e = ebase + p of position p gets
// the estimate, the raw count (the AND count, or for OR the ones of the OR)
// and the similarity `measure` (each output only if its pointer is set).
template <int W, int U, int G, bool OR>
__device__ __forceinline__ void bf_row_emit(const SkView& s, const uint64_t (&ru)[TcTeam<W, G>::words], int32_t du,
                                            uint32_t pcu, const int32_t* __restrict__ adj, int64_t beg,
                                            int64_t end, int lane, const double* __restrict__ tab, int64_t ebase,
                                            double* __restrict__ est_out, uint32_t* __restrict__ raw_out,
                                            float* __restrict__ sim_out, int measure) {
  constexpr int T = TcTeam<W, G>::value;
  constexpr int Q = TcTeam<W, G>::words;
  constexpr int NT = G / T;
  const int k = lane % T;
  const bool reads = k * Q < W;
  for (int64_t p0 = beg + lane / T; p0 < end; p0 += (int64_t)NT * U) {
    int32_t x[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int64_t p = p0 + (int64_t)j * NT;
      x[j] = p < end ? adj[p] : -1;
    }
    uint64_t rv[U][Q];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      if (x[j] >= 0 && reads) {
        const uint64_t* r = s.words + bf_row_offset(x[j], W) + k * Q;
#pragma unroll
        for (int i = 0; i < Q; ++i) rv[j][i] = r[i];
      } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) rv[j][i] = 0;
      }
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      uint32_t c = 0;
#pragma unroll
      for (int i = 0; i < Q; ++i) c += (uint32_t)__popcll(ru[i] & rv[j][i]);
      c = team_sum<T>(c);
      if (k == 0 && x[j] >= 0) {
        const int64_t e = ebase + p0 + (int64_t)j * NT;
        uint32_t raw = c;
        double est;
        if constexpr (OR) {
          raw = pcu + s.pc[x[j]] - c;
          est = ((double)du + (double)s.deg[x[j]]) + tab[raw];
        } else {
          est = tab[c];
        }
        if (est_out) est_out[e] = est;
        if (raw_out) raw_out[e] = raw;
        if (sim_out) sim_out[e] = (float)similarity_of(measure, est, du, s.deg[x[j]]);
      }
    }
  }
}

template <int W, int U, int G, bool OR>
__device__ __forceinline__ void bf_item_emit(const SkView& s, int32_t v, const int32_t* __restrict__ adj,
                                             int64_t beg, int64_t end, int lane, const double* __restrict__ tab,
                                             int64_t ebase, double* __restrict__ est_out,
                                             uint32_t* __restrict__ raw_out, float* __restrict__ sim_out,
                                             int measure) {
  uint64_t ru[TcTeam<W, G>::words];
  load_team_row<W, G>(s.words, v, lane % TcTeam<W, G>::value, ru);
  bf_row_emit<W, U, G, OR>(s, ru, s.deg[v], OR ? s.pc[v] : 0u, adj, beg, end, lane, tab, ebase, est_out, raw_out,
                           sim_out, measure);
}

// All upper edges over the triangle count's slab plan, with per-edge outputs
// at the edges' CSR order (edge upoff[v] + p - ustart[v] at position p).
template <int W, bool OR>
__global__ __launch_bounds__(kBlock) void k_bf_edges_slab(SlabPlan P, SkView s, const int32_t* __restrict__ off,
                                                          const int32_t* __restrict__ ustart,
                                                          const int32_t* __restrict__ adj,
                                                          const int64_t* __restrict__ upoff,
                                                          double* __restrict__ est_out, uint32_t* __restrict__ raw_out,
                                                          float* __restrict__ sim_out, int measure) {
  const bool whole = (int64_t)blockIdx.x >= P.slab_grid;
  const int x = (int)(blockIdx.x % kSlabs);
  const int64_t blk = whole ? (int64_t)blockIdx.x - P.slab_grid : (int64_t)(blockIdx.x / kSlabs);
  const int64_t n_chunks = whole ? 0 : P.n_chunks[x];
  const int64_t n_medium_blocks = whole ? 0 : (P.n_medium[x] + 3) / 4;
  if (!whole && blk >= slab_blocks(P, x)) return;
  extern __shared__ double tab[];
  for (uint32_t i = threadIdx.x; i <= s.size; i += kBlock) tab[i] = s.table[i];
  __syncthreads();
  constexpr int U = RowUnroll<W>::value;
  const size_t n = (size_t)s.n;
  const int tid = threadIdx.x;
  if (whole) {
    const int64_t idx = (blk * kBlock + tid) / kSlabWholeGroup;
    if (idx < P.n_whole) {
      const int32_t v = P.verts[P.whole_at + idx];
      bf_item_emit<W, U, kSlabWholeGroup, OR>(s, v, adj, ustart[v], off[v + 1], tid % kSlabWholeGroup, tab,
                                              upoff[v] - ustart[v], est_out, raw_out, sim_out, measure);
    }
  } else if (blk < n_chunks) {
    const int64_t c = P.chunk_at[x] + blk;
    const int32_t v = P.chunk_vertex[c];
    bf_item_emit<W, U, kBlock, OR>(s, v, adj, P.chunk_begin[c], P.chunk_end[c], tid, tab, upoff[v] - ustart[v],
                                   est_out, raw_out, sim_out, measure);
  } else if (blk - n_chunks < n_medium_blocks) {
    const int64_t idx = (blk - n_chunks) * (kBlock / kWave) + tid / kWave;
    if (idx < P.n_medium[x]) {
      const int32_t v = P.verts[P.medium_at[x] + idx];
      bf_item_emit<W, U, kWave, OR>(s, v, adj, slab_begin(ustart, P.split, n, x, v), slab_end(off, P.split, n, x, v),
                                    lane_id(), tab, upoff[v] - ustart[v], est_out, raw_out, sim_out, measure);
    }
  } else {
    const int64_t idx = ((blk - n_chunks - n_medium_blocks) * kBlock + tid) / kSlabLightGroup;
    if (idx < P.n_light[x]) {
      const int32_t v = P.verts[P.light_at[x] + idx];
      bf_item_emit<W, U, kSlabLightGroup, OR>(s, v, adj, slab_begin(ustart, P.split, n, x, v),
                                              slab_end(off, P.split, n, x, v), tid % kSlabLightGroup, tab,
                                              upoff[v] - ustart[v], est_out, raw_out, sim_out, measure);
    }
  }
}

// Block i < slab_grid serves slab x = i mod kSlabs (the XCD it runs on) and
// works on the (i / kSlabs)-th block of that slab's plan; the slab part is
// sized for the busiest slab and surplus blocks of the other slabs write a
// zero partial. Blocks from slab_grid on take the whole vertices.
// Work of one group of G lanes on the upper neighbours adj[beg, end) of v.
template <int W, int U, int G, bool OR>
__device__ __forceinline__ double bf_item(const SkView& s, int32_t v, const int32_t* __restrict__ adj, int64_t beg,
                                          int64_t end, int lane, const double* __restrict__ tab) {
  uint64_t ru[TcTeam<W, G>::words];
  load_team_row<W, G>(s.words, v, lane % TcTeam<W, G>::value, ru);
  return bf_row_sum<W, U, G, OR>(s, ru, OR ? s.deg[v] : 0, OR ? s.pc[v] : 0u, adj, beg, end, lane, tab);
}

template <int W, bool OR>
__global__ __launch_bounds__(kBlock) void k_bf_tc_slab(SlabPlan P, SkView s, const int32_t* __restrict__ off,
                                                       const int32_t* __restrict__ ustart,
                                                       const int32_t* __restrict__ adj, double* __restrict__ partials) {
  const bool whole = (int64_t)blockIdx.x >= P.slab_grid;
  const int x = (int)(blockIdx.x % kSlabs);
  const int64_t blk = whole ? (int64_t)blockIdx.x - P.slab_grid : (int64_t)(blockIdx.x / kSlabs);
  const int64_t n_chunks = whole ? 0 : P.n_chunks[x];
  const int64_t n_medium_blocks = whole ? 0 : (P.n_medium[x] + 3) / 4;
  if (!whole && blk >= slab_blocks(P, x)) {
    if (threadIdx.x == 0) partials[blockIdx.x] = 0.0;
    return;
  }
  extern __shared__ double tab[];
  __shared__ double red[kBlock / kWave];
  for (uint32_t i = threadIdx.x; i <= s.size; i += kBlock) tab[i] = s.table[i];
  __syncthreads();
  constexpr int U = RowUnroll<W>::value;
  const size_t n = (size_t)s.n;
  const int tid = threadIdx.x;
  double acc = 0.0;
  if (whole) {  // kSlabWholeGroup lanes per whole vertex, all its upper neighbours
    const int64_t idx = (blk * kBlock + tid) / kSlabWholeGroup;
    if (idx < P.n_whole) {
      const int32_t v = P.verts[P.whole_at + idx];
      acc = bf_item<W, U, kSlabWholeGroup, OR>(s, v, adj, ustart[v], off[v + 1], tid % kSlabWholeGroup, tab);
    }
  } else if (blk < n_chunks) {  // heavy chunk: the whole block
    const int64_t c = P.chunk_at[x] + blk;
    acc = bf_item<W, U, kBlock, OR>(s, P.chunk_vertex[c], adj, P.chunk_begin[c], P.chunk_end[c], tid, tab);
  } else if (blk - n_chunks < n_medium_blocks) {  // medium: one wave per item
    const int64_t idx = (blk - n_chunks) * (kBlock / kWave) + tid / kWave;
    if (idx < P.n_medium[x]) {
      const int32_t v = P.verts[P.medium_at[x] + idx];
      acc = bf_item<W, U, kWave, OR>(s, v, adj, slab_begin(ustart, P.split, n, x, v), slab_end(off, P.split, n, x, v),
                                     lane_id(), tab);
    }
  } else {  // light: kSlabLightGroup lanes per item
    const int64_t idx = ((blk - n_chunks - n_medium_blocks) * kBlock + tid) / kSlabLightGroup;
    if (idx < P.n_light[x]) {
      const int32_t v = P.verts[P.light_at[x] + idx];
      acc = bf_item<W, U, kSlabLightGroup, OR>(s, v, adj, slab_begin(ustart, P.split, n, x, v),
                                                slab_end(off, P.split, n, x, v), tid % kSlabLightGroup, tab);
    }
  }
  const double r = block_sum_256(acc, red);
  if (tid == 0) partials[blockIdx.x] = r;
}

// ---- k-hash MinHash: triangle count over the slab plan (Section 4.3) --------
//
// Same plan and tiers as the Bloom-filter kernel: the group owning v keeps
// sig_v in registers and walks the upper neighbours x from the CSR. A team of
// kKhTeam lanes reads sig_x side by side (K / kKhTeam slots each, 16-byte
// loads), counts the positions where both signatures hold the same element,
// and the counts meet in quad DPP adds. Lane 0 of the team adds the estimate
// s (d_v + d_x) / (k + s) in FP64, the same operations as the per-pair path,
// so every edge's estimate is bit-identical to it; each block writes one
// partial.
constexpr int kKhTeam = 4;

template <int K, int U, int G>
__device__ __forceinline__ double kh_item(const SkView& s, int32_t v, const int32_t* __restrict__ adj, int64_t beg,
                                          int64_t end, int lane) {
  static_assert(G % kKhTeam == 0 && K % (4 * kKhTeam) == 0, "whole teams, whole 16-byte loads");
  constexpr int T = kKhTeam;
  constexpr int Q4 = K / T / 4;  // 16-byte loads per lane and row
  constexpr int NT = G / T;      // teams in the group
  const int k = lane % T;
  uint4 mv[Q4];
  const uint4* pv = reinterpret_cast<const uint4*>(s.sig + (size_t)v * K) + k * Q4;
#pragma unroll
  for (int i = 0; i < Q4; ++i) mv[i] = pv[i];
  const int32_t dv = s.deg[v];
  double acc = 0.0;
  for (int64_t p0 = beg + lane / T; p0 < end; p0 += (int64_t)NT * U) {
    int32_t x[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int64_t p = p0 + (int64_t)j * NT;
      x[j] = p < end ? adj[p] : -1;
    }
    uint4 r[U][Q4];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      if (x[j] >= 0) {
        const uint4* px = reinterpret_cast<const uint4*>(s.sig + (size_t)x[j] * K) + k * Q4;
#pragma unroll
        for (int i = 0; i < Q4; ++i) r[j][i] = px[i];
      } else {
#pragma unroll
        for (int i = 0; i < Q4; ++i) r[j][i] = make_uint4(kBottom, kBottom, kBottom, kBottom);
      }
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      uint32_t c = 0;
#pragma unroll
      for (int i = 0; i < Q4; ++i) {
        const uint4 a = mv[i], b = r[j][i];
        c += (uint32_t)(a.x == b.x && a.x != kBottom) + (uint32_t)(a.y == b.y && a.y != kBottom) +
             (uint32_t)(a.z == b.z && a.z != kBottom) + (uint32_t)(a.w == b.w && a.w != kBottom);
      }
      c = team_sum<T>(c);
      if (k == 0 && x[j] >= 0) acc += minhash_estimate(c, (uint32_t)K, dv, s.deg[x[j]]);
    }
  }
  return acc;
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_kh_tc_slab(SlabPlan P, SkView s, const int32_t* __restrict__ off,
                                                       const int32_t* __restrict__ ustart,
                                                       const int32_t* __restrict__ adj, double* __restrict__ partials) {
  const bool whole = (int64_t)blockIdx.x >= P.slab_grid;
  const int x = (int)(blockIdx.x % kSlabs);
  const int64_t blk = whole ? (int64_t)blockIdx.x - P.slab_grid : (int64_t)(blockIdx.x / kSlabs);
  const int64_t n_chunks = whole ? 0 : P.n_chunks[x];
  const int64_t n_medium_blocks = whole ? 0 : (P.n_medium[x] + 3) / 4;
  if (!whole && blk >= slab_blocks(P, x)) {
    if (threadIdx.x == 0) partials[blockIdx.x] = 0.0;
    return;
  }
  __shared__ double red[kBlock / kWave];
  constexpr int U = K <= 32 ? 4 : 2;
  const size_t n = (size_t)s.n;
  const int tid = threadIdx.x;
  double acc = 0.0;
  if (whole) {
    const int64_t idx = (blk * kBlock + tid) / kSlabWholeGroup;
    if (idx < P.n_whole) {
      const int32_t v = P.verts[P.whole_at + idx];
      acc = kh_item<K, U, kSlabWholeGroup>(s, v, adj, ustart[v], off[v + 1], tid % kSlabWholeGroup);
    }
  } else if (blk < n_chunks) {
    const int64_t c = P.chunk_at[x] + blk;
    acc = kh_item<K, U, kBlock>(s, P.chunk_vertex[c], adj, P.chunk_begin[c], P.chunk_end[c], tid);
  } else if (blk - n_chunks < n_medium_blocks) {
    const int64_t idx = (blk - n_chunks) * (kBlock / kWave) + tid / kWave;
    if (idx < P.n_medium[x]) {
      const int32_t v = P.verts[P.medium_at[x] + idx];
      acc = kh_item<K, U, kWave>(s, v, adj, slab_begin(ustart, P.split, n, x, v), slab_end(off, P.split, n, x, v),
                                 lane_id());
    }
  } else {
    const int64_t idx = ((blk - n_chunks - n_medium_blocks) * kBlock + tid) / kSlabLightGroup;
    if (idx < P.n_light[x]) {
      const int32_t v = P.verts[P.light_at[x] + idx];
      acc = kh_item<K, U, kSlabLightGroup>(s, v, adj, slab_begin(ustart, P.split, n, x, v),
                                           slab_end(off, P.split, n, x, v), tid % kSlabLightGroup);
    }
  }
  const double r = block_sum_256(acc, red);
  if (tid == 0) partials[blockIdx.x] = r;
}

// ---- 1-hash MinHash: vertex-centric union counts (Section 4.4) ---------------
//
// The per-pair union walk costs one dependent load per step. Here a wave
// serves one vertex v at a time: the keys of M_v (ascending: a 1-hash
// signature lists its bottom-k IDs in key order) go to LDS once; for each
// neighbour u the wave loads M_u, element e in lane e mod 64, computes each
// element's key and finds by binary search over M_v's keys the number `lo` of
// smaller keys and whether the key itself is there. In the union walk element
// e of M_u comes after e elements of M_u and lo of M_v, of which the common
// ones (counted by a ballot prefix) appear once: its position is e + lo minus
// the common elements before it. The common elements, those among the first k
// positions, and the union size follow from ballots. Distinct IDs have
// distinct keys (odd multiplier, bijective mix), so equal keys are the same
// element. The counts equal the per-pair walk's exactly. For the KMV
// estimators the k-th smallest union key is either the key of the element of
// M_u at position k - 1, or, when there is none, the element of M_v after
// k - a + c - 1 others, a being the elements of M_u before position k - 1 and
// c the common ones among them. The ratio estimators at k <= 128 replace the
// key search by a lookup of M_u's IDs in a hash table of M_v's (below).

constexpr int kOhAhead = 4;      // neighbour rows in flight per wave, a wave per pair
constexpr int kOhHalfAhead = 2;  // neighbour rows in flight per half wave (k <= 32)
constexpr int kOhTabAhead = 2;      // neighbour rows per group, ID-table path, whole waves (two groups in flight)
constexpr int kOhTabHalfAhead = 1;  // the same per half wave (k <= 32)

template <int E>
__device__ __forceinline__ void oh_keys_to_lds(const SkView& s, int32_t v, uint32_t nv, uint64_t* keys) {
  const uint32_t* row = s.sig + (size_t)v * s.size;
  const int l = lane_id();
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const uint32_t e = (uint32_t)(j * kWave + l);
    if (e < nv) keys[e] = mh_key(s.a1, s.c1, row[e]);
  }
}

// The ratio estimators need, for each element of M_u, only whether it is in
// M_v and, if so, its index there: equal IDs are equal keys, and the common
// elements keep their relative order in both rows, so the union position of
// a common element e of M_u is e plus its index in M_v minus the common
// elements before it. For k <= 128 the wave therefore puts M_v's IDs in a
// bucketed hash table in LDS and looks each element of M_u up by ID: the
// neighbour rows are never hashed to keys nor searched by key, and the counts
// are the key walk's exactly. With E elements per lane (E = 1 for k <= 64,
// 2 for k <= 128) the table has 128 E buckets of four ID slots (half a slot
// per bucket on average when full) and a byte per slot with the element's
// index in M_v. An ID goes to the first bucket, from its hash bucket on, that
// has a free slot, so a lookup reads one bucket (one 16-byte LDS read, and
// the bucket's four index bytes as one word) and moves on only past a full
// bucket without the ID; at most 16 E buckets are full.
template <int E>
struct OhTable {
  static constexpr int kBuckets = 128 * E;
  static constexpr int kSlots = 4 * kBuckets;
  static constexpr int kWords = kSlots + kBuckets;  // 32-bit words: the ID slots, then the index bytes
  static constexpr int kShift = E == 1 ? 25 : 24;   // Fibonacci hashing to log2(kBuckets) bits
};
constexpr uint32_t kOhFree = 0xFFFFFFFFu;  // no vertex has this ID

template <int E>
__device__ __forceinline__ uint32_t oh_bucket_of(uint32_t id) {
  return (id * 0x9E3779B1u) >> OhTable<E>::kShift;
}

// Clear the wave's table, then insert M_v's nv <= 64 E IDs, element j * 64 + l
// in lane l.
template <int E>
__device__ __forceinline__ void oh_table_to_lds(const SkView& s, int32_t v, uint32_t nv, uint32_t* tab) {
  using T = OhTable<E>;
  const int l = lane_id();
  uint4* ids4 = reinterpret_cast<uint4*>(tab);
#pragma unroll
  for (int j = 0; j < T::kBuckets / kWave; ++j) ids4[j * kWave + l] = make_uint4(kOhFree, kOhFree, kOhFree, kOhFree);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const uint32_t e = (uint32_t)(j * kWave + l);
    if (e < nv) {
      const uint32_t id = s.sig[(size_t)v * s.size + e];
      uint32_t b = oh_bucket_of<E>(id);
      // at most 64 E of the slots are ever taken, so a free one is always found
      for (;;) {
        int q = 0;
        while (q < 4 && atomicCAS(tab + 4 * b + q, kOhFree, id) != kOhFree) ++q;
        if (q < 4) {
          reinterpret_cast<uint8_t*>(tab + T::kSlots)[4 * b + q] = (uint8_t)e;
          break;
        }
        b = (b + 1) & (T::kBuckets - 1);
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lookups: the slots of a bucket holding the ID, and whether a bucket has a
// free slot (which ends a search).
__device__ __forceinline__ uint32_t oh_hits(const uint4& q, uint32_t id) {
  return (uint32_t)(q.x == id) | ((uint32_t)(q.y == id) << 1) | ((uint32_t)(q.z == id) << 2) |
         ((uint32_t)(q.w == id) << 3);
}
__device__ __forceinline__ bool oh_open(const uint4& q) {
  return max(max(q.x, q.y), max(q.z, q.w)) == kOhFree;  // the free mark is the largest word
}
// The ID table serves the ratio estimators for k <= 128; the KMV estimators
// need the keys themselves and larger k keep the key search.
template <int E, bool KMV>
__host__ __device__ constexpr bool oh_by_table() {
  return !KMV && E <= 2;
}
// 64-bit LDS words a wave of the 1-hash kernels holds.
template <int E, bool KMV>
__host__ __device__ constexpr int oh_lds_words() {
  return oh_by_table<E, KMV>() ? OhTable<E>::kWords / 2 : kWave * E;
}

// Estimate for the pair (v, u) given M_v's nv keys in LDS and this lane's
// elements of M_u (x[j] = element j*64 + lane); the same in every lane. With
// HALF (k <= 32, E = 1) each half of the wave serves a pair of its own: lane
// l holds element l mod 32 of its half's M_u, ballots are masked to the half,
// and the result is the same in every lane of the half. du < 0 marks a half
// without a pair; its result is not used. Every lane takes every ballot and
// shuffle, so the halves never diverge around them.
template <int E, bool HALF, bool KMV>
__device__ __forceinline__ double oh_wave_estimate(const SkView& s, const uint64_t* keys_v, uint32_t nv, int32_t dv,
                                                   int32_t du, const uint32_t (&x)[E]) {
  static_assert(!HALF || E == 1, "half waves hold at most 32 elements");
  const uint32_t nu = du < 0 ? 0u : ((uint32_t)du < s.size ? (uint32_t)du : s.size);
  const int l = lane_id();
  const uint64_t hmask = HALF ? ((l & 32) ? 0xFFFFFFFF00000000ull : 0x00000000FFFFFFFFull) : ~0ull;
  const int base = HALF ? (l & 32) : 0;            // first lane of this lane's half
  const uint32_t le = (uint32_t)(l - base);        // element index within the half
  const uint64_t below = ((1ull << l) - 1ull) & hmask;  // lanes holding earlier elements of this batch
  uint32_t com = 0, comk = 0, a_k = 0, c_k = 0;
  uint64_t kth = ~0ull, max_u = 0;
  bool kth_in_u = false;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const uint32_t e = (uint32_t)(j * kWave) + le;
    bool found = false;
    uint32_t lo = 0;
    uint64_t key = 0;
    if (e < nu) {
      key = mh_key(s.a1, s.c1, x[j]);
      uint32_t hi = nv;  // lo: first position whose key is not below `key`
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (keys_v[mid] < key)
          lo = mid + 1;
        else
          hi = mid;
      }
      found = lo < nv && keys_v[lo] == key;
    }
    const uint64_t fb = __ballot(found) & hmask;
    const uint32_t before = com + (uint32_t)__popcll(fb & below);  // common elements ahead of e
    const bool first_k = found && e + lo - before < s.size;
    com += (uint32_t)__popcll(fb);
    comk += (uint32_t)__popcll(__ballot(first_k) & hmask);
    if constexpr (KMV) {
      const uint32_t pos = e + lo - before;  // union position of element e of M_u
      const uint64_t at = __ballot(e < nu && pos == s.size - 1) & hmask;
      const uint64_t kcand = (uint64_t)__shfl((unsigned long long)key, at ? __ffsll((long long)at) - 1 : l);
      if (at) {
        kth = kcand;
        kth_in_u = true;
      }
      a_k += (uint32_t)__popcll(__ballot(e < nu && pos < s.size - 1) & hmask);
      c_k += (uint32_t)__popcll(__ballot(e < nu && found && pos < s.size - 1) & hmask);
      const bool last_here = nu > 0 && (nu - 1) / kWave == (uint32_t)j;
      const uint64_t mcand =
          (uint64_t)__shfl((unsigned long long)key, last_here ? base + (int)((nu - 1) % kWave) : l);
      if (last_here) max_u = mcand;
    }
  }
  if constexpr (KMV) {
    const uint32_t uni = nu + nv - com;
    if (!kth_in_u && uni >= s.size) {
      const uint32_t iv = s.size - a_k + c_k - 1;  // index in M_v of the k-th union element
      kth = iv < nv ? keys_v[iv] : ~0ull;
    }
    return kmv_estimate(s.est == PG_EST_KMV, s.size, du, dv, nu, nv, uni, kth, max_u, nv ? keys_v[nv - 1] : 0ull);
  }
  if (s.est == PG_EST_MH_1HASH_LITERAL) return minhash_estimate(com, s.size, du, dv);
  const uint32_t uni = nu + nv - com;
  const uint32_t kp = uni < s.size ? uni : s.size;
  return minhash_estimate(uni >= s.size ? comk : com, kp, du, dv);
}

// Integer counts of the 1-hash ratio estimators for the pair (v, u), as in
// oh_wave_estimate: sc = the matches the estimator counts and kk its
// denominator (union reading: s and k' of the bottom-k' union; literal
// reading: |M_u cap M_v| and k). The same in every lane (of the half).
template <int E, bool HALF>
__device__ __forceinline__ void oh_wave_ratio_counts(const SkView& s, const uint64_t* keys_v, uint32_t nv, int32_t du,
                                                     const uint32_t (&x)[E], uint32_t& sc, uint32_t& kk) {
  static_assert(!HALF || E == 1, "half waves hold at most 32 elements");
  const uint32_t nu = du < 0 ? 0u : ((uint32_t)du < s.size ? (uint32_t)du : s.size);
  const int l = lane_id();
  const uint64_t hmask = HALF ? ((l & 32) ? 0xFFFFFFFF00000000ull : 0x00000000FFFFFFFFull) : ~0ull;
  const int base = HALF ? (l & 32) : 0;
  const uint32_t le = (uint32_t)(l - base);
  const uint64_t below = ((1ull << l) - 1ull) & hmask;
  uint32_t com = 0, comk = 0;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const uint32_t e = (uint32_t)(j * kWave) + le;
    bool found = false;
    uint32_t lo = 0;
    if (e < nu) {
      const uint64_t key = mh_key(s.a1, s.c1, x[j]);
      uint32_t hi = nv;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (keys_v[mid] < key)
          lo = mid + 1;
        else
          hi = mid;
      }
      found = lo < nv && keys_v[lo] == key;
    }
    const uint64_t fb = __ballot(found) & hmask;
    const uint32_t before = com + (uint32_t)__popcll(fb & below);
    const bool first_k = found && e + lo - before < s.size;
    com += (uint32_t)__popcll(fb);
    comk += (uint32_t)__popcll(__ballot(first_k) & hmask);
  }
  if (s.est == PG_EST_MH_1HASH_LITERAL) {
    sc = com;
    kk = s.size;
    return;
  }
  const uint32_t uni = nu + nv - com;
  kk = uni < s.size ? uni : s.size;
  sc = uni >= s.size ? comk : com;
}

// oh_wave_ratio_counts for k <= 128 over the ID table of M_v, for A
// neighbours at once (du[t] < 0: none): their bucket reads are issued
// together, then resolved. HALF needs E = 1.
template <bool HALF, int A, int E>
__device__ __forceinline__ void oh_table_ratio_counts(const SkView& s, const uint32_t* tab, uint32_t nv,
                                                      const int32_t (&du)[A], const uint32_t (&x)[A][E],
                                                      uint32_t (&sc)[A], uint32_t (&kk)[A]) {
  static_assert(!HALF || E == 1, "half waves hold at most 32 elements");
  using T = OhTable<E>;
  const int l = lane_id();
  const uint64_t hmask = HALF ? ((l & 32) ? 0xFFFFFFFF00000000ull : 0x00000000FFFFFFFFull) : ~0ull;
  const uint32_t le = (uint32_t)(l - (HALF ? (l & 32) : 0));
  const uint64_t below = ((1ull << l) - 1ull) & hmask;
  const uint4* ids4 = reinterpret_cast<const uint4*>(tab);
  const uint32_t* index4 = tab + T::kSlots;  // a bucket's four index bytes as one word
  uint32_t nu[A], b[A][E], hit[A][E], w[A][E];
  uint4 q[A][E];
#pragma unroll
  for (int t = 0; t < A; ++t) {
    nu[t] = du[t] < 0 ? 0u : ((uint32_t)du[t] < s.size ? (uint32_t)du[t] : s.size);
#pragma unroll
    for (int j = 0; j < E; ++j) {
      b[t][j] = oh_bucket_of<E>(x[t][j]);
      q[t][j] = ids4[b[t][j]];
      w[t][j] = index4[b[t][j]];
    }
  }
#pragma unroll
  for (int t = 0; t < A; ++t) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const bool mine = (uint32_t)(j * kWave) + le < nu[t];
      hit[t][j] = mine ? oh_hits(q[t][j], x[t][j]) : 0u;
      if (mine && hit[t][j] == 0u && !oh_open(q[t][j])) {  // a full bucket without the ID: rare
        do {
          b[t][j] = (b[t][j] + 1) & (T::kBuckets - 1);
          q[t][j] = ids4[b[t][j]];
          w[t][j] = index4[b[t][j]];
          hit[t][j] = oh_hits(q[t][j], x[t][j]);
        } while (hit[t][j] == 0u && !oh_open(q[t][j]));
      }
    }
  }
  uint32_t iv[A][E];
#pragma unroll
  for (int t = 0; t < A; ++t)
#pragma unroll
    for (int j = 0; j < E; ++j)
      iv[t][j] = hit[t][j] ? (w[t][j] >> (8u * (uint32_t)__builtin_ctz(hit[t][j]))) & 0xFFu : 0u;
#pragma unroll
  for (int t = 0; t < A; ++t) {
    uint32_t com = 0, comk = 0;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const uint32_t e = (uint32_t)(j * kWave) + le;
      const bool found = hit[t][j] != 0u;
      const uint64_t fb = __ballot(found) & hmask;
      const uint32_t before = com + (uint32_t)__popcll(fb & below);  // common elements ahead of this one
      const bool first_k = found && e + iv[t][j] - before < s.size;
      com += (uint32_t)__popcll(fb);
      comk += (uint32_t)__popcll(__ballot(first_k) & hmask);
    }
    // literal reading: |M_u cap M_v| of k; union reading: s of k'
    const bool lit = s.est == PG_EST_MH_1HASH_LITERAL;
    const uint32_t uni = nu[t] + nv - com;
    kk[t] = lit ? s.size : (uni < s.size ? uni : s.size);
    sc[t] = (lit || uni < s.size) ? com : comk;
  }
}

// The ratio estimate s/kk -> J/(1+J)(d_u + d_v) is FP64 work with divisions
// that every lane of the wave would repeat for every pair. Instead the pairs a
// wave evaluates are numbered in order; lane q mod 64 keeps the counts of
// pair q (written into that lane alone, s and kk packed in one word), and
// after every 64 pairs all lanes map their counts at once. Each estimate is
// the per-pair path's value; each lane adds its estimates in pair order and
// the lanes' sums meet in a fixed butterfly, so the total does not depend on
// scheduling. d_v is the item owner's, the same for all its pairs.
struct OhDeferred {
  int32_t dv;
  uint32_t counts = 0;  // lane q: s << 16 | kk of pair q (s, kk <= k <= 1024)
  int32_t du = 0;       // lane q: d_u of pair q
  uint32_t n = 0;       // pairs held, the same in every lane
  double acc = 0.0;
  __device__ explicit OhDeferred(int32_t dv_) : dv(dv_) {}
  __device__ __forceinline__ void flush() {
    if ((uint32_t)lane_id() < n) acc += minhash_estimate(counts >> 16, counts & 0xFFFFu, du, dv);
    n = 0;
  }
  // s_, kk_ and du_ are the same in every lane
  __device__ __forceinline__ void put(uint32_t s_, uint32_t kk_, int32_t du_) {
    const bool mine = (uint32_t)lane_id() == n;
    counts = mine ? ((s_ << 16) | kk_) : counts;
    du = mine ? du_ : du;
    if (++n == (uint32_t)kWave) flush();
  }
  __device__ __forceinline__ double total() {
    flush();
    return group_sum<kWave>(acc);
  }
};

// Sum of the estimates of (v, adj[p]) over p in [beg, end), one wave. For
// k <= 32 the two halves of the wave take neighbours p and p + 1 side by side;
// the result is then the sum of the two halves' sums, the same in every lane.
template <int E, bool HALF, bool KMV>
__device__ __forceinline__ double oh_wave_item(const SkView& s, int32_t v, const int32_t* __restrict__ adj,
                                               int64_t beg, int64_t end, uint64_t* keys) {
  constexpr bool TAB = oh_by_table<E, KMV>();
  const int32_t dv = s.deg[v];
  const uint32_t nv = (uint32_t)dv < s.size ? (uint32_t)dv : s.size;
  if constexpr (TAB) {
    oh_table_to_lds<E>(s, v, nv, reinterpret_cast<uint32_t*>(keys));
  } else {
    oh_keys_to_lds<E>(s, v, nv, keys);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  const int l = lane_id();
  double acc = 0.0;     // KMV: the same in every lane (of the half)
  OhDeferred df(dv);    // ratio estimators: deferred estimates
  if constexpr (HALF) {  // k <= 32 (the launch checks it): a separate kernel, so the wave-per-pair loop keeps its registers
    static_assert(E == 1, "half waves hold at most 32 elements");
    const int h = l >> 5;
    const uint32_t le = (uint32_t)(l & 31);
    if constexpr (!KMV) {
      // the ID-table path: as for whole waves, the next group's rows are
      // loaded (whole, without waiting for the degrees) during the lookups
      const uint32_t* tab = reinterpret_cast<const uint32_t*>(keys);
      const bool in_row = le < s.size;
      auto load = [&](int64_t p0, int32_t (&du)[kOhTabHalfAhead], uint32_t (&x)[kOhTabHalfAhead][1]) {
#pragma unroll
        for (int t = 0; t < kOhTabHalfAhead; ++t) {
          const int64_t p = p0 + 2 * t + h;
          const int32_t u = p < end ? adj[p] : -1;
          du[t] = u >= 0 ? s.deg[u] : -1;
          x[t][0] = (u >= 0 && in_row) ? s.sig[(size_t)u * s.size + le] : 0u;
        }
      };
      int32_t du[kOhTabHalfAhead], du_next[kOhTabHalfAhead];
      uint32_t x[kOhTabHalfAhead][1], x_next[kOhTabHalfAhead][1];
      if (beg < end) load(beg, du, x);
      for (int64_t p0 = beg; p0 < end; p0 += 2 * kOhTabHalfAhead) {
        const bool more = p0 + 2 * kOhTabHalfAhead < end;
        if (more) load(p0 + 2 * kOhTabHalfAhead, du_next, x_next);
        uint32_t sc[kOhTabHalfAhead], kk[kOhTabHalfAhead];
        oh_table_ratio_counts<true, kOhTabHalfAhead, 1>(s, tab, nv, du, x, sc, kk);
#pragma unroll
        for (int t = 0; t < kOhTabHalfAhead; ++t) {
          const int32_t du0 = __shfl(du[t], 0), du1 = __shfl(du[t], kWave / 2);
          const uint32_t s0 = (uint32_t)__shfl((int)sc[t], 0), k0 = (uint32_t)__shfl((int)kk[t], 0);
          const uint32_t s1 = (uint32_t)__shfl((int)sc[t], kWave / 2), k1 = (uint32_t)__shfl((int)kk[t], kWave / 2);
          if (du0 >= 0) df.put(s0, k0, du0);
          if (du1 >= 0) df.put(s1, k1, du1);
        }
        if (more) {
#pragma unroll
          for (int t = 0; t < kOhTabHalfAhead; ++t) {
            du[t] = du_next[t];
            x[t][0] = x_next[t][0];
          }
        }
      }
      return df.total();
    } else {
      for (int64_t p0 = beg; p0 < end; p0 += 2 * kOhHalfAhead) {
        int32_t du[kOhHalfAhead];
        uint32_t x[kOhHalfAhead][1];
#pragma unroll
        for (int t = 0; t < kOhHalfAhead; ++t) {
          const int64_t p = p0 + 2 * t + h;
          const int32_t u = p < end ? adj[p] : -1;
          du[t] = u >= 0 ? s.deg[u] : -1;
          const uint32_t nu = u < 0 ? 0u : ((uint32_t)du[t] < s.size ? (uint32_t)du[t] : s.size);
          x[t][0] = le < nu ? s.sig[(size_t)u * s.size + le] : 0u;
        }
#pragma unroll
        for (int t = 0; t < kOhHalfAhead; ++t) {
          const double est = oh_wave_estimate<1, true, KMV>(s, keys, nv, dv, du[t], x[t]);
          if (du[t] >= 0) acc += est;
        }
      }
      return __shfl(acc, 0) + __shfl(acc, kWave / 2);
    }
  } else {
  if constexpr (TAB) {
    // kOhTabAhead neighbours at a time, the next group's degrees and rows loaded
    // while this group is looked up; a row is loaded whole (k slots) without
    // waiting for the degree, which masks the lanes afterwards
    const uint32_t* tab = reinterpret_cast<const uint32_t*>(keys);
    bool in_row[E];  // element j * 64 + l is a slot of the rows
#pragma unroll
    for (int j = 0; j < E; ++j) in_row[j] = (uint32_t)(j * kWave + l) < s.size;
    auto load = [&](int64_t p0, int32_t (&du)[kOhTabAhead], uint32_t (&x)[kOhTabAhead][E]) {
#pragma unroll
      for (int t = 0; t < kOhTabAhead; ++t) {
        const int32_t u = p0 + t < end ? adj[p0 + t] : -1;
        du[t] = u >= 0 ? s.deg[u] : -1;
#pragma unroll
        for (int j = 0; j < E; ++j)
          x[t][j] = (u >= 0 && in_row[j]) ? s.sig[(size_t)u * s.size + j * kWave + l] : 0u;
      }
    };
    int32_t du[kOhTabAhead], du_next[kOhTabAhead];
    uint32_t x[kOhTabAhead][E], x_next[kOhTabAhead][E];
    if (beg < end) load(beg, du, x);
    for (int64_t p0 = beg; p0 < end; p0 += kOhTabAhead) {
      const bool more = p0 + kOhTabAhead < end;
      if (more) load(p0 + kOhTabAhead, du_next, x_next);
      uint32_t sc[kOhTabAhead], kk[kOhTabAhead];
      oh_table_ratio_counts<false, kOhTabAhead, E>(s, tab, nv, du, x, sc, kk);
#pragma unroll
      for (int t = 0; t < kOhTabAhead; ++t)
        if (du[t] >= 0) df.put(sc[t], kk[t], du[t]);
      if (more) {
#pragma unroll
        for (int t = 0; t < kOhTabAhead; ++t) {
          du[t] = du_next[t];
#pragma unroll
          for (int j = 0; j < E; ++j) x[t][j] = x_next[t][j];
        }
      }
    }
    return df.total();
  } else {
  // kOhAhead neighbours at a time: their degrees and rows are loaded before
  // any of them is evaluated
  for (int64_t p0 = beg; p0 < end; p0 += kOhAhead) {
    int32_t du[kOhAhead];
    uint32_t x[kOhAhead][E];
#pragma unroll
    for (int t = 0; t < kOhAhead; ++t) {
      const int32_t u = p0 + t < end ? adj[p0 + t] : -1;
      du[t] = u >= 0 ? s.deg[u] : -1;
      const uint32_t nu = u < 0 ? 0u : ((uint32_t)du[t] < s.size ? (uint32_t)du[t] : s.size);
      const uint32_t* row = s.sig + (size_t)(u < 0 ? 0 : u) * s.size;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const uint32_t e = (uint32_t)(j * kWave + l);
        x[t][j] = e < nu ? row[e] : 0u;
      }
    }
#pragma unroll
    for (int t = 0; t < kOhAhead; ++t) {
      if (du[t] < 0) continue;
      if constexpr (KMV) {
        acc += oh_wave_estimate<E, false, KMV>(s, keys, nv, dv, du[t], x[t]);
      } else {
        uint32_t sc, kk;
        oh_wave_ratio_counts<E, false>(s, keys, nv, du[t], x[t], sc, kk);
        df.put(sc, kk, du[t]);
      }
    }
  }
  if constexpr (KMV) return acc;
  return df.total();
  }
  }
}

// Blocks of slab x when every light or medium item gets one wave.
__host__ __device__ inline int64_t oh_slab_blocks(const SlabPlan& p, int x) {
  return p.n_chunks[x] + (p.n_medium[x] + 3) / 4 + (p.n_light[x] + 3) / 4;
}

// Triangle count over the slab plan: block i < grid_slabs serves slab i mod
// kSlabs; a heavy chunk is split among the block's four waves in contiguous
// quarters. Blocks from grid_slabs on take the whole vertices. One partial per wave.
template <int E, bool HALF, bool KMV>
__global__ __launch_bounds__(kBlock) void k_oh_tc_slab(SlabPlan P, SkView s, const int32_t* __restrict__ off,
                                                       const int32_t* __restrict__ ustart,
                                                       const int32_t* __restrict__ adj, int64_t grid_slabs,
                                                       double* __restrict__ partials) {
  __shared__ __align__(16) uint64_t keys[kBlock / kWave][oh_lds_words<E, KMV>()];
  const int w = threadIdx.x / kWave;
  const size_t n = (size_t)s.n;
  double acc = 0.0;
  if ((int64_t)blockIdx.x >= grid_slabs) {  // whole vertices, one wave each
    const int64_t idx = ((int64_t)blockIdx.x - grid_slabs) * (kBlock / kWave) + w;
    if (idx < P.n_whole) {
      const int32_t v = P.verts[P.whole_at + idx];
      acc = oh_wave_item<E, HALF, KMV>(s, v, adj, ustart[v], off[v + 1], keys[w]);
    }
  } else {
    const int x = (int)(blockIdx.x % kSlabs);
    const int64_t blk = blockIdx.x / kSlabs;
    const int64_t nmb = (P.n_medium[x] + 3) / 4;
    if (blk < P.n_chunks[x]) {
      const int64_t c = P.chunk_at[x] + blk;
      const int64_t cb = P.chunk_begin[c], ce = P.chunk_end[c];
      const int64_t q = (ce - cb + 3) / 4;
      const int64_t b0 = cb + w * q;
      const int64_t e0 = b0 + q < ce ? b0 + q : ce;
      if (b0 < e0) acc = oh_wave_item<E, HALF, KMV>(s, P.chunk_vertex[c], adj, b0, e0, keys[w]);
    } else if (blk - P.n_chunks[x] < nmb) {
      const int64_t idx = (blk - P.n_chunks[x]) * (kBlock / kWave) + w;
      if (idx < P.n_medium[x]) {
        const int32_t v = P.verts[P.medium_at[x] + idx];
        acc = oh_wave_item<E, HALF, KMV>(s, v, adj, slab_begin(ustart, P.split, n, x, v), slab_end(off, P.split, n, x, v),
                              keys[w]);
      }
    } else {
      const int64_t idx = (blk - P.n_chunks[x] - nmb) * (kBlock / kWave) + w;
      if (idx < P.n_light[x]) {
        const int32_t v = P.verts[P.light_at[x] + idx];
        acc = oh_wave_item<E, HALF, KMV>(s, v, adj, slab_begin(ustart, P.split, n, x, v), slab_end(off, P.split, n, x, v),
                              keys[w]);
      }
    }
  }
  if (lane_id() == 0) partials[(int64_t)blockIdx.x * (kBlock / kWave) + w] = acc;
}

// Clustering coefficient over the full-neighbourhood plan: light vertices
// (natural order) and medium ones get a wave, heavy vertices are split into
// chunks whose four waves write one partial sum per chunk (combined below).
template <int E, bool HALF, bool KMV>
__global__ __launch_bounds__(kBlock) void k_oh_cc_plan(PlanView P, SkView s, const int32_t* __restrict__ off,
                                                       const int32_t* __restrict__ adj, float* __restrict__ cc,
                                                       double* __restrict__ vsum, double* __restrict__ part) {
  __shared__ __align__(16) uint64_t keys[kBlock / kWave][oh_lds_words<E, KMV>()];
  __shared__ double red[kBlock / kWave];
  const int w = threadIdx.x / kWave;
  const int64_t blk = blockIdx.x;
  if (blk < P.n_chunks) {
    const int64_t cb = P.chunk_begin[blk], ce = P.chunk_end[blk];
    const int64_t q = (ce - cb + 3) / 4;
    const int64_t b0 = cb + w * q;
    const int64_t e0 = b0 + q < ce ? b0 + q : ce;
    double acc = 0.0;
    if (b0 < e0) acc = oh_wave_item<E, HALF, KMV>(s, P.chunk_vertex[blk], adj, b0, e0, keys[w]);
    if (lane_id() == 0) red[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blk] = (red[0] + red[1]) + (red[2] + red[3]);
    return;
  }
  const int64_t mb = blk - P.n_chunks;
  int32_t v = -1;
  if (mb < P.n_medium_blocks) {
    const int64_t idx = mb * (kBlock / kWave) + w;
    if (idx < P.n_medium) v = P.medium[idx];
  } else {
    const int64_t idx = (mb - P.n_medium_blocks) * (kBlock / kWave) + w;
    if (idx < P.n_light) {
      v = P.light ? P.light[idx] : (int32_t)idx;
      if (off[v + 1] - off[v] > kLightMax) v = -1;  // a medium or heavy vertex in natural order
    }
  }
  if (v < 0) return;
  const double tot = oh_wave_item<E, HALF, KMV>(s, v, adj, off[v], off[v + 1], keys[w]);
  if (lane_id() == 0) {
    const int32_t d = s.deg[v];
    cc[v] = (float)(d >= 2 ? tot / ((double)d * ((double)d - 1.0)) : 0.0);
    if (vsum) vsum[v] = tot;
  }
}

// Heavy vertices: chunk partials summed in chunk order.
__global__ void k_cc_combine(PlanView P, const double* __restrict__ part, int64_t n_heavy,
                                const int32_t* __restrict__ deg, float* __restrict__ cc, double* __restrict__ vsum) {
  const int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (h >= n_heavy) return;
  const int32_t c0 = P.heavy_first[h], c1 = P.heavy_first[h + 1];
  const int32_t v = P.chunk_vertex[c0];
  double tot = 0.0;
  for (int32_t c = c0; c < c1; ++c) tot += part[c];
  const int32_t d = deg[v];
  cc[v] = (float)(d >= 2 ? tot / ((double)d * ((double)d - 1.0)) : 0.0);
  if (vsum) vsum[v] = tot;
}

template <typename F>
int oh_dispatch_e(uint32_t k, F&& launch) {
  const uint32_t e = (k + kWave - 1) / kWave;
  if (k <= (uint32_t)kWave / 2) return launch(std::integral_constant<int, 1>(), std::true_type());  // half waves
  if (e <= 1) return launch(std::integral_constant<int, 1>(), std::false_type());
  if (e <= 2) return launch(std::integral_constant<int, 2>(), std::false_type());
  if (e <= 4) return launch(std::integral_constant<int, 4>(), std::false_type());
  if (e <= 8) return launch(std::integral_constant<int, 8>(), std::false_type());
  return launch(std::integral_constant<int, 16>(), std::false_type());
}

// ---- clustering coefficient over XCD slabs of all of N_v ---------------------
//
// The triangle count's slab plan built over all arcs: block i < slab_grid
// works on slab i mod kSlabs, so each XCD gathers the rows of an eighth of
// the vertices. A vertex with at most kSliceMin arcs ("whole") is summed by
// one group of kSlabWholeGroup lanes, which writes its coefficient. A sliced
// vertex's items write their sums to part[x * n_sliced + rank[v]] (zero where
// it has no arcs in slab x) and its heavy chunks to chunk_part; then
// k_cc_slab_combine adds them in slab order, then chunk order. F is the
// sketch kind's per-item sum (the triangle count's item over all of N_v).
template <int W, bool OR>
struct BfCcItem {
  static constexpr bool kTable = true;  // the estimator table staged in LDS
  template <int G>
  __device__ static double sum(const SkView& s, int32_t v, const int32_t* __restrict__ adj, int64_t beg, int64_t end,
                               int lane, const double* __restrict__ tab) {
    return bf_item<W, RowUnroll<W>::value, G, OR>(s, v, adj, beg, end, lane, tab);
  }
};

template <int K>
struct KhCcItem {
  static constexpr bool kTable = false;
  template <int G>
  __device__ static double sum(const SkView& s, int32_t v, const int32_t* __restrict__ adj, int64_t beg, int64_t end,
                               int lane, const double* __restrict__) {
    return kh_item<K, (K <= 32 ? 4 : 2), G>(s, v, adj, beg, end, lane);
  }
};

template <class F>
__global__ __launch_bounds__(kBlock) void k_cc_slab(SlabPlan P, SkView s, const int32_t* __restrict__ off,
                                                    const int32_t* __restrict__ adj, float* __restrict__ cc,
                                                    double* __restrict__ vsum, double* __restrict__ part,
                                                    double* __restrict__ chunk_part) {
  const bool whole = (int64_t)blockIdx.x >= P.slab_grid;
  const int x = (int)(blockIdx.x % kSlabs);
  const int64_t blk = whole ? (int64_t)blockIdx.x - P.slab_grid : (int64_t)(blockIdx.x / kSlabs);
  const int64_t n_chunks = whole ? 0 : P.n_chunks[x];
  const int64_t n_medium_blocks = whole ? 0 : (P.n_medium[x] + 3) / 4;
  if (!whole && blk >= slab_blocks(P, x)) return;
  extern __shared__ double tab[];
  __shared__ double red[kBlock / kWave];
  if constexpr (F::kTable) {
    for (uint32_t i = threadIdx.x; i <= s.size; i += kBlock) tab[i] = s.table[i];
    __syncthreads();
  }
  const size_t n = (size_t)s.n;
  const int tid = threadIdx.x;
  if (whole) {
    const int64_t idx = (blk * kBlock + tid) / kSlabWholeGroup;
    int32_t v = -1;
    double acc = 0.0;
    if (idx < P.n_whole) {
      v = P.verts[P.whole_at + idx];
      acc = F::template sum<kSlabWholeGroup>(s, v, adj, off[v], off[v + 1], tid % kSlabWholeGroup, tab);
    }
    const double tot = group_sum<kSlabWholeGroup>(acc);
    if (v >= 0 && tid % kSlabWholeGroup == 0) {
      const int32_t d = s.deg[v];
      cc[v] = (float)(d >= 2 ? tot / ((double)d * ((double)d - 1.0)) : 0.0);
      if (vsum) vsum[v] = tot;
    }
  } else if (blk < n_chunks) {  // heavy chunk: the whole block
    const int64_t c = P.chunk_at[x] + blk;
    const double acc =
        F::template sum<kBlock>(s, P.chunk_vertex[c], adj, P.chunk_begin[c], P.chunk_end[c], tid, tab);
    const double r = block_sum_256(acc, red);
    if (tid == 0) chunk_part[c] = r;
  } else if (blk - n_chunks < n_medium_blocks) {  // medium: one wave per item
    const int64_t idx = (blk - n_chunks) * (kBlock / kWave) + tid / kWave;
    int32_t v = -1;
    double acc = 0.0;
    if (idx < P.n_medium[x]) {
      v = P.verts[P.medium_at[x] + idx];
      acc = F::template sum<kWave>(s, v, adj, slab_begin(off, P.split, n, x, v), slab_end(off, P.split, n, x, v),
                                   lane_id(), tab);
    }
    const double tot = group_sum<kWave>(acc);
    if (v >= 0 && lane_id() == 0) part[(size_t)x * (size_t)P.n_sliced + (size_t)P.rank[v]] = tot;
  } else {  // light: kSlabLightGroup lanes per item
    const int64_t idx = ((blk - n_chunks - n_medium_blocks) * kBlock + tid) / kSlabLightGroup;
    int32_t v = -1;
    double acc = 0.0;
    if (idx < P.n_light[x]) {
      v = P.verts[P.light_at[x] + idx];
      acc = F::template sum<kSlabLightGroup>(s, v, adj, slab_begin(off, P.split, n, x, v),
                                             slab_end(off, P.split, n, x, v), tid % kSlabLightGroup, tab);
    }
    const double tot = group_sum<kSlabLightGroup>(acc);
    if (v >= 0 && tid % kSlabLightGroup == 0) part[(size_t)x * (size_t)P.n_sliced + (size_t)P.rank[v]] = tot;
  }
}

// Coefficients of the sliced vertices from their item and chunk sums, and of
// the vertices without arcs (0); whole vertices were written by k_cc_slab.
__global__ void k_cc_slab_combine(SlabPlan P, int32_t n, const int32_t* __restrict__ deg,
                                  const double* __restrict__ part, const double* __restrict__ chunk_part,
                                  float* __restrict__ cc, double* __restrict__ vsum) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t r = P.rank[v];
  const int32_t d = deg[v];
  if (r < 0) {
    if (d == 0) {
      cc[v] = 0.0f;
      if (vsum) vsum[v] = 0.0;
    }
    return;
  }
  double tot = 0.0;
#pragma unroll
  for (int x = 0; x < kSlabs; ++x) tot += part[(size_t)x * (size_t)P.n_sliced + (size_t)r];
  for (int32_t i = P.chunk_ptr[r]; i < P.chunk_ptr[r + 1]; ++i) tot += chunk_part[P.chunk_list[i]];
  cc[v] = (float)(d >= 2 ? tot / ((double)d * ((double)d - 1.0)) : 0.0);
  if (vsum) vsum[v] = tot;
}


__global__ void k_make_table(double* __restrict__ t, uint32_t B, uint32_t b, int est) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c > B) return;
  const double Bd = (double)B, bd = (double)b;
  const double ct = (double)(c == B ? c - 1 : c);  // Appendix C: B~_1 = B_1 - [B_1 = B]
  double r;
  switch (est) {
    case PG_EST_BF_AND:
      r = -(Bd / bd) * log(1.0 - ct / Bd);
      break;
    case PG_EST_BF_L:
      r = (double)c / bd;
      break;
    case PG_EST_BF_PAPAPETROU:
      r = log(1.0 - ct / Bd) / (bd * log(1.0 - 1.0 / Bd));
      break;
    default:  // PG_EST_BF_OR: the logarithmic term, added to |X| + |Y|
      r = (Bd / bd) * log(1.0 - ct / Bd);
      break;
  }
  t[c] = r;
}

// Dispatch on (kind, W): Bloom filters get an instantiation per word count up
// to 16 words; wider filters and MinHash use the general path.
#define PG_DISPATCH(sk, LAUNCH)                    \
  do {                                             \
    if ((sk)->kind == PG_BF) {                     \
      switch ((sk)->W) {                           \
        case 1: LAUNCH(PG_BF, 1); break;           \
        case 2: LAUNCH(PG_BF, 2); break;           \
        case 3: LAUNCH(PG_BF, 3); break;           \
        case 4: LAUNCH(PG_BF, 4); break;           \
        case 5: LAUNCH(PG_BF, 5); break;           \
        case 6: LAUNCH(PG_BF, 6); break;           \
        case 7: LAUNCH(PG_BF, 7); break;           \
        case 8: LAUNCH(PG_BF, 8); break;           \
        case 9: LAUNCH(PG_BF, 9); break;           \
        case 10: LAUNCH(PG_BF, 10); break;         \
        case 11: LAUNCH(PG_BF, 11); break;         \
        case 12: LAUNCH(PG_BF, 12); break;         \
        case 13: LAUNCH(PG_BF, 13); break;         \
        case 14: LAUNCH(PG_BF, 14); break;         \
        case 15: LAUNCH(PG_BF, 15); break;         \
        case 16: LAUNCH(PG_BF, 16); break;         \
        default: LAUNCH(PG_BF, 0); break;          \
      }                                            \
    } else if ((sk)->kind == PG_MH_KHASH) {        \
      LAUNCH(PG_MH_KHASH, 0);                      \
    } else {                                       \
      LAUNCH(PG_MH_1HASH, 0);                      \
    }                                              \
  } while (0)

}  // namespace

SkView make_view(const pg_sketches* sk, int est) {
  SkView v{};
  v.kind = sk->kind;
  v.est = est;
  v.size = sk->size;
  v.b = sk->b;
  v.W = sk->W;
  v.n = sk->g->n;
  v.words = sk->words;
  v.pc = sk->pc;
  v.sig = sk->sig;
  v.table = bf_table(sk, est);
  v.deg = sk->rows->deg;  // sizes of the sketched sets: d_v, or d+_v for oriented rows
  if (sk->kind == PG_MH_1HASH) hash_constants(PG_MH_1HASH, sk->seed, 1, &v.a1, &v.c1);
  return v;
}

int check_estimator(const pg_sketches* sk, int est) {
  const bool bf = est == PG_EST_BF_AND || est == PG_EST_BF_L || est == PG_EST_BF_OR || est == PG_EST_BF_PAPAPETROU;
  if (sk->kind == PG_BF && bf) return PG_OK;
  if (sk->kind == PG_MH_KHASH && est == PG_EST_MH_KHASH) return PG_OK;
  if (sk->kind == PG_MH_1HASH && (est == PG_EST_MH_1HASH || est == PG_EST_MH_1HASH_LITERAL || est == PG_EST_KMV ||
                                  est == PG_EST_KMV_SKETCH_SIZES))
    return PG_OK;
  return fail(PG_E_INVALID, "estimator does not match the sketch kind");
}

int64_t chunk_count(int64_t npairs) { return (npairs + kChunk - 1) / kChunk; }

int fill_table(double* table, uint32_t B, uint32_t b, int est, hipStream_t s) {
  const uint32_t entries = B + 1;
  ProfScope ps(s, "table");
  hipLaunchKernelGGL(k_make_table, dim3((entries + kBlock - 1) / kBlock), dim3(kBlock), 0, s, table, B, b, est);
  PG_LAUNCH_CHECK();
  return PG_OK;
}

int fill_tables(pg_sketches* sk, hipStream_t s) {
  if (sk->kind != PG_BF) return PG_OK;
  for (int i = 0; i < kBfTables; ++i)
    PG_TRY(fill_table(sk->table + (size_t)i * (sk->size + 1), sk->size, sk->b, PG_EST_BF_AND + i, s));
  return PG_OK;
}

const double* bf_table(const pg_sketches* sk, int est) {
  if (sk->kind != PG_BF || est < PG_EST_BF_AND || est > PG_EST_BF_PAPAPETROU) return nullptr;
  return sk->table + (size_t)(est - PG_EST_BF_AND) * (sk->size + 1);
}

int estimate_pairs(const pg_sketches* sk, int est, const int32_t* u, const int32_t* v, int64_t npairs,
                   double* est_out, uint32_t* raw_out, float* sim_out, int measure, hipStream_t s) {
  PG_TRY(check_estimator(sk, est));
  if (sim_out && sk->oriented) return fail(PG_E_UNSUPPORTED, kOrientedNeedsNv);
  if (sim_out && (measure < PG_SIM_COMMON || measure > PG_SIM_TOTAL))
    return fail(PG_E_INVALID, "unknown similarity measure");
  if (npairs <= 0) return PG_OK;
  const SkView view = make_view(sk, est);
  const pg_graph* g = sk->g;
  if (sk->kind == PG_BF && sk->W <= 16 && u == g->eu && v == g->ev && npairs == g->m) {
    // all upper edges (the caller passed none): walk the triangle count's
    // XCD slab plan and write each edge's values at its CSR position
    PG_TRY(graph_slabs(const_cast<pg_graph*>(g), s));
    const SlabPlan& P = g->slabs;
    const int64_t nblk = slab_plan_blocks(P);
    if (nblk > (int64_t)(UINT32_MAX / kBlock)) return fail(PG_E_UNSUPPORTED, "graph too large for one launch");
    const size_t shmem = sizeof(double) * ((size_t)sk->size + 1);
    ProfScope ps(s, "edges");
#define PG_EDS(WW)                                                                                                     \
  do {                                                                                                                 \
    if (est == PG_EST_BF_OR)                                                                                           \
      hipLaunchKernelGGL((k_bf_edges_slab<WW, true>), dim3((unsigned)nblk), dim3(kBlock), shmem, s, P, view, g->off,   \
                         g->ustart, g->adj, (const int64_t*)g->upoff, est_out, raw_out, sim_out, measure);             \
    else                                                                                                               \
      hipLaunchKernelGGL((k_bf_edges_slab<WW, false>), dim3((unsigned)nblk), dim3(kBlock), shmem, s, P, view, g->off,  \
                         g->ustart, g->adj, (const int64_t*)g->upoff, est_out, raw_out, sim_out, measure);             \
  } while (0)
    if (nblk > 0) {
      switch (sk->W) {
        case 1: PG_EDS(1); break;
        case 2: PG_EDS(2); break;
        case 3: PG_EDS(3); break;
        case 4: PG_EDS(4); break;
        case 5: PG_EDS(5); break;
        case 6: PG_EDS(6); break;
        case 7: PG_EDS(7); break;
        case 8: PG_EDS(8); break;
        case 9: PG_EDS(9); break;
        case 10: PG_EDS(10); break;
        case 11: PG_EDS(11); break;
        case 12: PG_EDS(12); break;
        case 13: PG_EDS(13); break;
        case 14: PG_EDS(14); break;
        case 15: PG_EDS(15); break;
        default: PG_EDS(16); break;
      }
      PG_LAUNCH_CHECK();
    }
#undef PG_EDS
    return PG_OK;
  }
  const unsigned grid = grid_for(npairs, kBlock, 65536);
  ProfScope ps(s, "pairs");
#define PG_LAUNCH_PAIRS(KIND, WT)                                                                                   \
  hipLaunchKernelGGL((k_pairs<KIND, WT>), dim3(grid), dim3(kBlock), 0, s, view, u, v, npairs, est_out, raw_out, \
                     sim_out, measure)
  PG_DISPATCH(sk, PG_LAUNCH_PAIRS);
#undef PG_LAUNCH_PAIRS
  PG_LAUNCH_CHECK();
  return PG_OK;
}

int estimate_jp(const pg_sketches* sk, int est, int measure, double tau, uint8_t* keep, unsigned long long* d_kept,
                hipStream_t s) {
  PG_TRY(check_estimator(sk, est));
  if (sk->oriented) return fail(PG_E_UNSUPPORTED, kOrientedNeedsNv);
  if (measure < PG_SIM_COMMON || measure > PG_SIM_TOTAL) return fail(PG_E_INVALID, "unknown similarity measure");
  PG_TRY(fill_u64((uint64_t*)d_kept, 0, 1, s));
  const pg_graph* g = sk->g;
  if (g->m <= 0) return PG_OK;
  const SkView view = make_view(sk, est);
  // a few blocks per CU: every block adds its count to one shared counter,
  // and device-scope atomics on one address serialise
  const unsigned grid = grid_for(g->m, kBlock, (int64_t)std::max(1, g->ctx->num_cus) * kCountBlocksPerCu);
  const int32_t* eu = g->eu;
  const int32_t* ev = g->ev;
  const int64_t m = g->m;
  ProfScope ps(s, "jarvis_patrick");
#define PG_LAUNCH_JP(KIND, WT) \
  hipLaunchKernelGGL((k_pairs_jp<KIND, WT>), dim3(grid), dim3(kBlock), 0, s, view, eu, ev, m, measure, tau, keep, d_kept)
  PG_DISPATCH(sk, PG_LAUNCH_JP);
#undef PG_LAUNCH_JP
  PG_LAUNCH_CHECK();
  return PG_OK;
}

int estimate_sum(const pg_sketches* sk, int est, const int32_t* u, const int32_t* v, int64_t npairs, double* chunks,
                 hipStream_t s) {
  PG_TRY(check_estimator(sk, est));
  const int64_t nchunks = chunk_count(npairs);
  if (nchunks <= 0) return PG_OK;
  const SkView view = make_view(sk, est);
  const unsigned grid = (unsigned)std::min<int64_t>(nchunks, 65536);
  ProfScope ps(s, "pairs_sum");
#define PG_LAUNCH_SUM(KIND, WT) \
  hipLaunchKernelGGL((k_pairs_sum<KIND, WT>), dim3(grid), dim3(kBlock), 0, s, view, u, v, npairs, chunks)
  PG_DISPATCH(sk, PG_LAUNCH_SUM);
#undef PG_LAUNCH_SUM
  PG_LAUNCH_CHECK();
  return PG_OK;
}

int estimate_tc(const pg_sketches* sk, int est, double* d_out, hipStream_t s, const TcWorkspace* ws) {
  PG_TRY(check_estimator(sk, est));
  // partial sums (and the tiles of their sum): in the caller's workspace, or
  // allocated for this call
  auto get_parts = [&](int64_t count, double** parts, double** tiles) -> int {
    *parts = *tiles = nullptr;
    if (!ws) return dmalloc((void**)parts, sizeof(double) * (size_t)count, s);
    if (count + sum_chunks_tiles(count) > ws->doubles)
      return fail(PG_E_UNSUPPORTED, "triangle count: " + std::to_string(count + sum_chunks_tiles(count)) +
                                        " partial sums exceed the fixed workspace of " + std::to_string(ws->doubles));
    *parts = ws->ptr;
    *tiles = ws->ptr + count;
    return PG_OK;
  };
  auto put_parts = [&](double* parts) { return ws ? PG_OK : dfree(parts, s); };
  auto plan = [&]() -> int {
    if (ws && !sk->g->slabs.split)
      return fail(PG_E_UNSUPPORTED, "the graph's triangle-count plan is not built yet: it is built (and allocated) by "
                                    "the first pg_tc or pg_tc_async call on a sketch set of this graph");
    return graph_slabs(const_cast<pg_graph*>(sk->g), s);
  };
  const pg_graph* g = sk->g;
  // every kernel below sums the estimate over the m edges, each once: a triangle
  // contributes three edges over N_v, one over N+_v (Listing "lst:tc")
  const double divisor = sk->oriented ? 1.0 : 3.0;
  if (sk->kind == PG_BF && sk->W <= 16 && g->n > 0) {
    PG_TRY(plan());
    const SlabPlan& P = g->slabs;
    const int64_t nblk = std::max<int64_t>(slab_plan_blocks(P), 1);
    if (nblk > (int64_t)(UINT32_MAX / kBlock)) return fail(PG_E_UNSUPPORTED, "graph too large for one triangle-count launch");
    double *partials, *tiles;
    PG_TRY(get_parts(nblk, &partials, &tiles));
    const SkView view = make_view(sk, est);
    const size_t shmem = sizeof(double) * ((size_t)sk->size + 1);
    {
      ProfScope ps(s, "bf_tc");
#define PG_TCP(WW)                                                                                                    \
  do {                                                                                                                \
    if (est == PG_EST_BF_OR)                                                                                          \
      hipLaunchKernelGGL((k_bf_tc_slab<WW, true>), dim3((unsigned)nblk), dim3(kBlock), shmem, s, P, view, g->off,     \
                         g->ustart, g->adj, partials);                                                                \
    else                                                                                                              \
      hipLaunchKernelGGL((k_bf_tc_slab<WW, false>), dim3((unsigned)nblk), dim3(kBlock), shmem, s, P, view, g->off,    \
                         g->ustart, g->adj, partials);                                                                \
  } while (0)
      switch (sk->W) {
        case 1: PG_TCP(1); break;
        case 2: PG_TCP(2); break;
        case 3: PG_TCP(3); break;
        case 4: PG_TCP(4); break;
        case 5: PG_TCP(5); break;
        case 6: PG_TCP(6); break;
        case 7: PG_TCP(7); break;
        case 8: PG_TCP(8); break;
        case 9: PG_TCP(9); break;
        case 10: PG_TCP(10); break;
        case 11: PG_TCP(11); break;
        case 12: PG_TCP(12); break;
        case 13: PG_TCP(13); break;
        case 14: PG_TCP(14); break;
        case 15: PG_TCP(15); break;
        default: PG_TCP(16); break;
      }
#undef PG_TCP
      PG_LAUNCH_CHECK();
    }
    PG_TRY(sum_chunks(partials, nblk, divisor, d_out, s, tiles));
    return put_parts(partials);
  }
  if (sk->kind == PG_MH_KHASH && (sk->size == 16 || sk->size == 32 || sk->size == 64) && g->n > 0) {
    PG_TRY(plan());
    const SlabPlan& P = g->slabs;
    const int64_t nblk = std::max<int64_t>(slab_plan_blocks(P), 1);
    if (nblk > (int64_t)(UINT32_MAX / kBlock)) return fail(PG_E_UNSUPPORTED, "graph too large for one triangle-count launch");
    double *partials, *tiles;
    PG_TRY(get_parts(nblk, &partials, &tiles));
    const SkView view = make_view(sk, est);
    {
      ProfScope ps(s, "kh_tc");
      if (sk->size == 16)
        hipLaunchKernelGGL(k_kh_tc_slab<16>, dim3((unsigned)nblk), dim3(kBlock), 0, s, P, view, g->off, g->ustart, g->adj,
                           partials);
      else if (sk->size == 32)
        hipLaunchKernelGGL(k_kh_tc_slab<32>, dim3((unsigned)nblk), dim3(kBlock), 0, s, P, view, g->off, g->ustart, g->adj,
                           partials);
      else
        hipLaunchKernelGGL(k_kh_tc_slab<64>, dim3((unsigned)nblk), dim3(kBlock), 0, s, P, view, g->off, g->ustart, g->adj,
                           partials);
      PG_LAUNCH_CHECK();
    }
    PG_TRY(sum_chunks(partials, nblk, divisor, d_out, s, tiles));
    return put_parts(partials);
  }
  if (sk->kind == PG_MH_1HASH && is_onehash_union(est) && g->n > 0) {
    PG_TRY(plan());
    const SlabPlan& P = g->slabs;
    int64_t busiest = 0;
    for (int x = 0; x < kSlabs; ++x) busiest = std::max(busiest, oh_slab_blocks(P, x));
    const int64_t grid_slabs = busiest * kSlabs;
    const int64_t nblk = std::max<int64_t>(grid_slabs + (P.n_whole + 3) / 4, 1);
    if (nblk > (int64_t)(UINT32_MAX / kBlock)) return fail(PG_E_UNSUPPORTED, "graph too large for one launch");
    const int64_t nparts = nblk * (kBlock / kWave);
    double *partials, *tiles;
    PG_TRY(get_parts(nparts, &partials, &tiles));
    const SkView view = make_view(sk, est);
    {
      ProfScope ps(s, "oh_tc");
      PG_TRY(oh_dispatch_e(sk->size, [&](auto e, auto half) {
        constexpr int EE = decltype(e)::value;
        constexpr bool HH = decltype(half)::value;
        if (is_minhash_ratio(est))
          hipLaunchKernelGGL((k_oh_tc_slab<EE, HH, false>), dim3((unsigned)nblk), dim3(kBlock), 0, s, P, view, g->off,
                             g->ustart, g->adj, grid_slabs, partials);
        else
          hipLaunchKernelGGL((k_oh_tc_slab<EE, HH, true>), dim3((unsigned)nblk), dim3(kBlock), 0, s, P, view, g->off,
                             g->ustart, g->adj, grid_slabs, partials);
        PG_LAUNCH_CHECK();
        return PG_OK;
      }));
    }
    PG_TRY(sum_chunks(partials, nparts, divisor, d_out, s, tiles));
    return put_parts(partials);
  }
  // general path: one lane per upper edge, fixed chunks
  const int64_t nchunks = std::max<int64_t>(chunk_count(g->m), 1);
  double *chunks, *tiles;
  PG_TRY(get_parts(nchunks, &chunks, &tiles));
  PG_TRY(fill_u64((uint64_t*)chunks, 0, nchunks, s));
  if (g->m > 0) PG_TRY(estimate_sum(sk, est, g->eu, g->ev, g->m, chunks, s));
  PG_TRY(sum_chunks(chunks, nchunks, divisor, d_out, s, tiles));
  return put_parts(chunks);
}

int estimate_cc(const pg_sketches* sk, int est, float* cc, double* vsum, hipStream_t s) {
  PG_TRY(check_estimator(sk, est));
  if (sk->oriented) return fail(PG_E_UNSUPPORTED, kOrientedNeedsNv);
  const pg_graph* g = sk->g;
  const SkView view = make_view(sk, est);
  ProfScope ps(s, "cc");
  if (sk->kind == PG_MH_1HASH && is_onehash_union(est)) {
    const VertexPlan& P = g->plan_all;
    const PlanView pv = plan_view(P);
    const int64_t nblk = P.n_chunks + pv.n_medium_blocks + (P.n_light + 3) / 4;
    if (nblk <= 0) return PG_OK;
    if (nblk > (int64_t)(UINT32_MAX / kBlock)) return fail(PG_E_UNSUPPORTED, "graph too large for one launch");
    double* part = nullptr;
    PG_TRY(dmalloc((void**)&part, sizeof(double) * (size_t)std::max<int64_t>(P.n_chunks, 1), s));
    PG_TRY(oh_dispatch_e(sk->size, [&](auto e, auto half) {
      constexpr int EE = decltype(e)::value;
      constexpr bool HH = decltype(half)::value;
      if (is_minhash_ratio(est))
        hipLaunchKernelGGL((k_oh_cc_plan<EE, HH, false>), dim3((unsigned)nblk), dim3(kBlock), 0, s, pv, view, g->off,
                           g->adj, cc, vsum, part);
      else
        hipLaunchKernelGGL((k_oh_cc_plan<EE, HH, true>), dim3((unsigned)nblk), dim3(kBlock), 0, s, pv, view, g->off,
                           g->adj, cc, vsum, part);
      PG_LAUNCH_CHECK();
      return PG_OK;
    }));
    if (P.n_heavy > 0) {
      hipLaunchKernelGGL(k_cc_combine, dim3((unsigned)((P.n_heavy + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, pv,
                         (const double*)part, P.n_heavy, g->deg, cc, vsum);
      PG_LAUNCH_CHECK();
    }
    return dfree(part, s);
  }
  // the slab plan over all of N_v: part (8 sums per sliced vertex, zero where
  // it has no item) and chunk sums, the launch, then the per-vertex combine
  auto slab_cc = [&](size_t shmem, auto launch) -> int {
    PG_TRY(graph_slabs_all(const_cast<pg_graph*>(g), s));
    const SlabPlan& P = g->slabs_all;
    const int64_t nblk = slab_plan_blocks(P);
    if (nblk > (int64_t)(UINT32_MAX / kBlock)) return fail(PG_E_UNSUPPORTED, "graph too large for one launch");
    int64_t n_chunks = 0;
    for (int x = 0; x < kSlabs; ++x) n_chunks += P.n_chunks[x];
    const int64_t n_part = (int64_t)kSlabs * P.n_sliced;
    double* part = nullptr;
    PG_TRY(dmalloc((void**)&part, sizeof(double) * (size_t)std::max<int64_t>(n_part + n_chunks, 1), s));
    double* chunk_part = part + n_part;
    if (n_part > 0) PG_TRY(fill_u64(reinterpret_cast<uint64_t*>(part), 0, n_part, s));  // 0.0 where v has no item
    if (nblk > 0) {
      launch(P, dim3((unsigned)nblk), shmem, part, chunk_part);
      PG_LAUNCH_CHECK();
    }
    if (g->n > 0) {
      hipLaunchKernelGGL(k_cc_slab_combine, dim3((unsigned)((g->n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, P,
                         g->n, (const int32_t*)g->deg, (const double*)part, (const double*)chunk_part, cc, vsum);
      PG_LAUNCH_CHECK();
    }
    return dfree(part, s);
  };
  if (sk->kind == PG_MH_KHASH && (sk->size == 16 || sk->size == 32 || sk->size == 64)) {
    return slab_cc(0, [&](const SlabPlan& P, dim3 grid, size_t shmem, double* part, double* chunk_part) {
      if (sk->size == 16)
        hipLaunchKernelGGL(k_cc_slab<KhCcItem<16>>, grid, dim3(kBlock), shmem, s, P, view, g->off, g->adj, cc, vsum,
                           part, chunk_part);
      else if (sk->size == 32)
        hipLaunchKernelGGL(k_cc_slab<KhCcItem<32>>, grid, dim3(kBlock), shmem, s, P, view, g->off, g->adj, cc, vsum,
                           part, chunk_part);
      else
        hipLaunchKernelGGL(k_cc_slab<KhCcItem<64>>, grid, dim3(kBlock), shmem, s, P, view, g->off, g->adj, cc, vsum,
                           part, chunk_part);
    });
  }
  if (sk->kind == PG_BF && sk->W <= 16) {
    return slab_cc(sizeof(double) * ((size_t)sk->size + 1),
                   [&](const SlabPlan& P, dim3 grid, size_t shmem, double* part, double* chunk_part) {
#define PG_CCS(WW)                                                                                                 \
  do {                                                                                                             \
    if (est == PG_EST_BF_OR)                                                                                       \
      hipLaunchKernelGGL((k_cc_slab<BfCcItem<WW, true>>), grid, dim3(kBlock), shmem, s, P, view, g->off, g->adj,    \
                         cc, vsum, part, chunk_part);                                                              \
    else                                                                                                           \
      hipLaunchKernelGGL((k_cc_slab<BfCcItem<WW, false>>), grid, dim3(kBlock), shmem, s, P, view, g->off, g->adj,   \
                         cc, vsum, part, chunk_part);                                                              \
  } while (0)
                     switch (sk->W) {
                       case 1: PG_CCS(1); break;
                       case 2: PG_CCS(2); break;
                       case 3: PG_CCS(3); break;
                       case 4: PG_CCS(4); break;
                       case 5: PG_CCS(5); break;
                       case 6: PG_CCS(6); break;
                       case 7: PG_CCS(7); break;
                       case 8: PG_CCS(8); break;
                       case 9: PG_CCS(9); break;
                       case 10: PG_CCS(10); break;
                       case 11: PG_CCS(11); break;
                       case 12: PG_CCS(12); break;
                       case 13: PG_CCS(13); break;
                       case 14: PG_CCS(14); break;
                       case 15: PG_CCS(15); break;
                       default: PG_CCS(16); break;
                     }
#undef PG_CCS
                   });
  }
  for (int bin = 0; bin < kNumBins; ++bin) {
    const int64_t cnt = g->bin_start[bin + 1] - g->bin_start[bin];
    if (cnt <= 0) continue;
    const int32_t* verts = g->bin_verts + g->bin_start[bin];
    const int G = kBinGroup[bin];
    const unsigned grid = (unsigned)((cnt * G + kBlock - 1) / kBlock);
#define PG_LAUNCH_CC_G(KIND, WT, GG) \
  hipLaunchKernelGGL((k_cc<KIND, WT, GG>), dim3(grid), dim3(kBlock), 0, s, view, g->off, g->adj, verts, cnt, cc, vsum)
#define PG_LAUNCH_CC(KIND, WT)        \
  do {                                \
    if (G == 4)                       \
      PG_LAUNCH_CC_G(KIND, WT, 4);    \
    else if (G == 16)                 \
      PG_LAUNCH_CC_G(KIND, WT, 16);   \
    else if (G == 64)                 \
      PG_LAUNCH_CC_G(KIND, WT, 64);   \
    else                              \
      PG_LAUNCH_CC_G(KIND, WT, 256);  \
  } while (0)
    PG_DISPATCH(sk, PG_LAUNCH_CC);
#undef PG_LAUNCH_CC
#undef PG_LAUNCH_CC_G
    PG_LAUNCH_CHECK();
  }
  return PG_OK;
}

int noalloc_scratch(int device, double** ptr, int64_t* doubles) {
  // device addresses of the array, one per device, each looked up once with
  // that device current (the caller has made `device` current)
  static std::mutex mu;
  static double* addr[64] = {};
  if (device < 0 || device >= 64) return fail(PG_E_INVALID, "device ordinal out of range for the fixed workspace");
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(PG_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    addr[device] = (double*)p;
  }
  *ptr = addr[device];
  *doubles = kScratchDoubles;
  return PG_OK;
}

}  // namespace pg
