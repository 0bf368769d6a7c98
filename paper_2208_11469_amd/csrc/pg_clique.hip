// 4-clique counting (Listing "lst:fcl"): with the degree order R of the
// triangle count, for every oriented edge (u, v), v in N+_u, the third
// vertices of its triangles are C3 = N+_u cap N+_v, and every w in C3
// contributes |N+_w cap C3|; each 4-clique is counted once, at its three
// lowest-ranked vertices. The count |N+_w cap C3| is exact (binary search of
// x in N+_w) or, from Bloom filters of the oriented sets, the number of x in
// C3 ranked above w (the only elements N+_w can hold) that pass the
// membership query of the filter of N+_w (Section 2.4: all b bits set; false
// positives only).
//
// One wave per oriented edge, edges dealt round-robin to the waves of a
// persistent grid. The wave builds C3 in its LDS slice: lanes take 64
// elements of the shorter list at a time, binary-search them in the longer
// list, and a ballot appends the hits in ID order (with their degrees, for
// the rank test, and with filters the first hash function's bit index, so
// each element is hashed once per edge rather than once per pair). For
// |C3| <= 64 the |C3| (|C3| - 1) / 2 unordered pairs are dealt to the lanes,
// the lower-ranked element of each pair playing w; otherwise the wave takes
// one w at a time (with filters its row is staged in LDS) and the lanes
// stride over x, testing those ranked above w. Counts are integers: the result does not depend on
// scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pg_device.h"
#include "pg_internal.h"

namespace pg {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;
constexpr int kMaxLdsBytes = 128 * 1024;
constexpr int kRowInts = 32;  // staged filter row: up to 16 words

struct CliqueFilters {
  const uint64_t* words;  // line-packed rows of the filters of N+_v
  const uint64_t* ha;
  const uint64_t* hc;
  uint32_t B, W, b;
};

// LDS visibility among the lanes of one wave.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// x in the ascending list[0, len)?
__device__ __forceinline__ bool sorted_contains(const int32_t* __restrict__ list, int32_t len, int32_t x) {
  int32_t lo = 0, hi = len;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (list[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo < len && list[lo] == x;
}

// Rows of the filters: WT the row width as a compile-time constant (1..16,
// line-packed rows), or 0 for rows wider than 16 words (dense: row v at v * W).
template <int WT>
__device__ __forceinline__ const uint64_t* filter_row(const CliqueFilters& f, int32_t w) {
  return f.words + (WT > 0 ? bf_row_offset(w, (uint32_t)WT) : (size_t)w * f.W);
}

// Membership of x in the filter `row`: bit i0 (the first hash function's,
// precomputed) and the bits of the other b - 1 functions all set.
__device__ __forceinline__ uint32_t member(const uint64_t* row, const CliqueFilters& f, int32_t x, uint32_t i0) {
  if (!((row[i0 >> 6] >> (i0 & 63u)) & 1ull)) return 0;
  for (uint32_t h = 1; h < f.b; ++h) {
    const uint32_t idx = bf_index(f.ha[h], f.hc[h], (uint32_t)x, f.B);
    if (!((row[idx >> 6] >> (idx & 63u)) & 1ull)) return 0;
  }
  return 1;
}

__device__ __forceinline__ bool ranked_below(int32_t w, int32_t dw, int32_t x, int32_t dx) {
  return dw < dx || (dw == dx && w < x);
}

// WT = -1: exact count; otherwise filters of row width WT (see filter_row).
// LDS slice of a wave: [staged row: kRowInts] [ids: cap] [degrees: cap]
// [first bit indices: cap, filters only]; cap is even, so slices stay 8-byte
// aligned.
template <int WT>
__global__ __launch_bounds__(kBlock) void k_four_cliques(const int32_t* __restrict__ poff,
                                                         const int32_t* __restrict__ padj,
                                                         const int32_t* __restrict__ parc_src, int64_t m,
                                                         const int32_t* __restrict__ deg, int32_t cap, CliqueFilters f,
                                                         unsigned long long* __restrict__ count) {
  constexpr bool kBf = WT >= 0;
  constexpr int kArrays = kBf ? 3 : 2;
  extern __shared__ int32_t lds[];
  __shared__ unsigned long long block_count;
  if (threadIdx.x == 0) block_count = 0;
  __syncthreads();
  const int wave = (int)threadIdx.x / kWave;
  const int lane = lane_id();
  int32_t* slice = lds + (size_t)wave * ((size_t)kRowInts + (size_t)kArrays * cap);
  uint64_t* rowbuf = reinterpret_cast<uint64_t*>(slice);
  int32_t* ids = slice + kRowInts;
  int32_t* dg = ids + cap;
  uint32_t* hx = reinterpret_cast<uint32_t*>(dg + cap);  // filters only
  unsigned long long mine = 0;
  const int64_t nwaves = (int64_t)gridDim.x * kWaves;
  for (int64_t e = (int64_t)blockIdx.x * kWaves + wave; e < m; e += nwaves) {
    const int32_t u = parc_src[e], v = padj[e];
    const int32_t* A = padj + poff[u];
    int32_t na = poff[u + 1] - poff[u];
    const int32_t* L = padj + poff[v];
    int32_t nl = poff[v + 1] - poff[v];
    if (na > nl) {
      const int32_t* t = A;
      A = L;
      L = t;
      const int32_t tn = na;
      na = nl;
      nl = tn;
    }
    // C3 = A cap L in ID order; |C3| <= na <= cap
    int32_t s = 0;
    for (int32_t base = 0; base < na; base += kWave) {
      const int32_t i = base + lane;
      int32_t a = 0;
      bool hit = false;
      if (i < na) {
        a = A[i];
        hit = sorted_contains(L, nl, a);
      }
      const uint64_t ball = __ballot(hit);
      if (hit) {
        const int32_t pos = s + (int32_t)__popcll(ball & ((1ull << lane) - 1ull));
        ids[pos] = a;
        dg[pos] = deg[a];
        if constexpr (kBf) hx[pos] = bf_index(f.ha[0], f.hc[0], (uint32_t)a, f.B);
      }
      s += (int32_t)__popcll(ball);
    }
    wave_sync();
    if (s >= 2) {
      if (s <= kWave) {
        // the s (s - 1) / 2 unordered pairs {i, j} of C3, dealt to the lanes;
        // w is the lower-ranked element (N+_w holds only vertices ranked above w)
        const int32_t npairs = s * (s - 1) / 2;
        for (int32_t p = lane; p < npairs; p += kWave) {
          // p = j (j - 1) / 2 + i with 0 <= i < j
          int32_t j = (int32_t)((1.0f + sqrtf(1.0f + 8.0f * (float)p)) * 0.5f);
          while (j * (j - 1) / 2 > p) --j;
          while ((j + 1) * j / 2 <= p) ++j;
          const int32_t i = p - j * (j - 1) / 2;
          const bool i_low = ranked_below(ids[i], dg[i], ids[j], dg[j]);
          const int32_t wi = i_low ? i : j, xi = i_low ? j : i;
          const int32_t w = ids[wi], x = ids[xi];
          if constexpr (kBf) {
            mine += member(filter_row<WT>(f, w), f, x, hx[xi]);
          } else {
            const int32_t b0 = poff[w];
            mine += sorted_contains(padj + b0, poff[w + 1] - b0, x) ? 1u : 0u;
          }
        }
      } else {
        for (int32_t wi = 0; wi < s; ++wi) {
          const int32_t w = ids[wi], dw = dg[wi];
          const uint64_t* row = nullptr;
          if constexpr (kBf) {
            if constexpr (WT > 0) {
              if (lane < WT) rowbuf[lane] = filter_row<WT>(f, w)[lane];
              wave_sync();
              row = rowbuf;
            } else {
              row = filter_row<WT>(f, w);
            }
          }
          for (int32_t xi = lane; xi < s; xi += kWave) {
            const int32_t x = ids[xi];
            if (!ranked_below(w, dw, x, dg[xi])) continue;
            if constexpr (kBf) {
              mine += member(row, f, x, hx[xi]);
            } else {
              const int32_t b0 = poff[w];
              mine += sorted_contains(padj + b0, poff[w + 1] - b0, x) ? 1u : 0u;
            }
          }
          if constexpr (WT > 0) wave_sync();  // before the next row overwrites the staged one
        }
      }
    }
    wave_sync();  // the next edge overwrites this wave's slice
  }
  if (mine) atomicAdd(&block_count, mine);
  __syncthreads();
  if (threadIdx.x == 0 && block_count) atomicAdd(count, block_count);
}

// ---- sketch intersections: |N+_w cap C3| from two filters -------------------
//
// The estimate of Listing "lst:fcl" with a sketch intersection per w: the
// wave builds C3 as above and, in the same pass, the filter of C3 in its LDS
// slice (B bits, the b hash functions of the sketch set, set with LDS
// atomics); every w in C3 then takes one lane, which reads the filter row of
// N+_w and counts the ones of its AND (or OR) with the filter of C3. The
// estimator table (B + 1 entries) sits in LDS. Each lane adds its estimates in
// a fixed order and every block writes one partial, so the FP64 result does
// not depend on scheduling.
template <int WT, bool OR>
__global__ __launch_bounds__(kBlock) void k_four_cliques_filters(const int32_t* __restrict__ poff,
                                                                 const int32_t* __restrict__ padj,
                                                                 const int32_t* __restrict__ parc_src, int64_t m,
                                                                 int32_t cap, CliqueFilters f,
                                                                 const double* __restrict__ table,
                                                                 double* __restrict__ partials) {
  extern __shared__ double tab[];  // [estimator table: B + 1] then the wave slices
  __shared__ double red[kWaves];
  const uint32_t W = WT > 0 ? (uint32_t)WT : f.W;
  for (uint32_t i = threadIdx.x; i <= f.B; i += kBlock) tab[i] = table[i];
  const int wave = (int)threadIdx.x / kWave;
  const int lane = lane_id();
  // wave slice: [filter of C3: W words] [ids: cap], cap even
  uint64_t* fc = reinterpret_cast<uint64_t*>(tab + f.B + 1) + (size_t)wave * ((size_t)W + (size_t)cap / 2);
  uint32_t* fc32 = reinterpret_cast<uint32_t*>(fc);
  int32_t* ids = reinterpret_cast<int32_t*>(fc + W);
  __syncthreads();
  double acc = 0.0;
  const int64_t nwaves = (int64_t)gridDim.x * kWaves;
  for (int64_t e = (int64_t)blockIdx.x * kWaves + wave; e < m; e += nwaves) {
    const int32_t u = parc_src[e], v = padj[e];
    const int32_t* A = padj + poff[u];
    int32_t na = poff[u + 1] - poff[u];
    const int32_t* L = padj + poff[v];
    int32_t nl = poff[v + 1] - poff[v];
    if (na > nl) {
      const int32_t* t = A;
      A = L;
      L = t;
      const int32_t tn = na;
      na = nl;
      nl = tn;
    }
    for (uint32_t i = (uint32_t)lane; i < 2 * W; i += kWave) fc32[i] = 0;
    wave_sync();
    int32_t s = 0;
    for (int32_t base = 0; base < na; base += kWave) {
      const int32_t i = base + lane;
      int32_t a = 0;
      bool hit = false;
      if (i < na) {
        a = A[i];
        hit = sorted_contains(L, nl, a);
      }
      const uint64_t ball = __ballot(hit);
      if (hit) {
        ids[s + (int32_t)__popcll(ball & ((1ull << lane) - 1ull))] = a;
        for (uint32_t h = 0; h < f.b; ++h) {
          const uint32_t idx = bf_index(f.ha[h], f.hc[h], (uint32_t)a, f.B);
          atomicOr(&fc32[idx >> 5], 1u << (idx & 31u));  // bit t: bit t & 63 of word t >> 6
        }
      }
      s += (int32_t)__popcll(ball);
    }
    wave_sync();
    for (int32_t i = lane; i < s; i += kWave) {
      const int32_t w = ids[i];
      const uint64_t* row = filter_row<WT>(f, w);
      uint32_t c = 0;
      if constexpr (WT > 0) {
        uint64_t r[WT];
#pragma unroll
        for (int j = 0; j < WT; ++j) r[j] = row[j];
#pragma unroll
        for (int j = 0; j < WT; ++j) c += (uint32_t)__popcll(OR ? (r[j] | fc[j]) : (r[j] & fc[j]));
      } else {
        for (uint32_t j = 0; j < W; ++j) c += (uint32_t)__popcll(OR ? (row[j] | fc[j]) : (row[j] & fc[j]));
      }
      if constexpr (OR)
        acc += ((double)(poff[w + 1] - poff[w]) + (double)s) + tab[c];
      else
        acc += tab[c];
    }
    wave_sync();  // the next edge clears this wave's slice
  }
  const double r = block_sum_256(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

}  // namespace

// The 4-clique estimate from sketch intersections into d_out[0] (device FP64):
// est is PG_EST_BF_AND, _L or _PAPAPETROU (a function of the ones of the AND)
// or PG_EST_BF_OR (|N+_w| + |C3| and the ones of the OR).
int four_cliques_estimate(const pg_sketches* sk, int est, double* d_out, hipStream_t s) {
  if (est != PG_EST_BF_AND && est != PG_EST_BF_L && est != PG_EST_BF_OR && est != PG_EST_BF_PAPAPETROU)
    return fail(PG_E_INVALID, "4-clique estimates take a Bloom-filter estimator");
  pg_graph* g = sk->g;
  PG_TRY(graph_oriented(g, s));
  PG_TRY(fill_u64((uint64_t*)d_out, 0, 1, s));  // 0.0
  if (g->m <= 0) return PG_OK;
  const int32_t cap = (std::max(1, g->oriented->max_degree) + 1) & ~1;
  const size_t shmem =
      sizeof(double) * ((size_t)sk->size + 1) + sizeof(uint64_t) * ((size_t)sk->W + (size_t)cap / 2) * kWaves;
  if (shmem > (size_t)kMaxLdsBytes)
    return fail(PG_E_UNSUPPORTED, "4-cliques: the filter size and the largest oriented degree exceed the on-chip buffers");
  CliqueFilters f{sk->words, sk->ha, sk->hc, sk->size, sk->W, sk->b};
  const unsigned grid = (unsigned)std::max<int64_t>(
      1, std::min<int64_t>((g->m + kWaves - 1) / kWaves, (int64_t)std::max(1, g->ctx->num_cus) * 8));
  double* partials = nullptr;
  PG_TRY(dmalloc((void**)&partials, sizeof(double) * grid, s));
  {
    ProfScope ps(s, "four_cliques_filters");
#define PG_CKF(WW)                                                                                                \
  do {                                                                                                            \
    if (est == PG_EST_BF_OR)                                                                                      \
      hipLaunchKernelGGL((k_four_cliques_filters<WW, true>), dim3(grid), dim3(kBlock), shmem, s, g->poff, g->padj, \
                         g->parc_src, g->m, cap, f, bf_table(sk, est), partials);                          \
    else                                                                                                          \
      hipLaunchKernelGGL((k_four_cliques_filters<WW, false>), dim3(grid), dim3(kBlock), shmem, s, g->poff,        \
                         g->padj, g->parc_src, g->m, cap, f, bf_table(sk, est), partials);                 \
  } while (0)
    switch (sk->W) {
      case 1: PG_CKF(1); break;
      case 2: PG_CKF(2); break;
      case 3: PG_CKF(3); break;
      case 4: PG_CKF(4); break;
      case 5: PG_CKF(5); break;
      case 6: PG_CKF(6); break;
      case 7: PG_CKF(7); break;
      case 8: PG_CKF(8); break;
      case 9: PG_CKF(9); break;
      case 10: PG_CKF(10); break;
      case 11: PG_CKF(11); break;
      case 12: PG_CKF(12); break;
      case 13: PG_CKF(13); break;
      case 14: PG_CKF(14); break;
      case 15: PG_CKF(15); break;
      case 16: PG_CKF(16); break;
      default: PG_CKF(0); break;  // rows wider than 16 words are dense
    }
#undef PG_CKF
    PG_LAUNCH_CHECK();
  }
  PG_TRY(sum_chunks(partials, grid, 1.0, d_out, s));
  return dfree(partials, s);
}

// The 4-clique count into d_count[0]: exact (sk == nullptr) or with Bloom
// filters of the oriented sets.
int four_cliques(pg_graph* g, const pg_sketches* sk, unsigned long long* d_count, hipStream_t s) {
  PG_TRY(graph_oriented(g, s));
  PG_TRY(fill_u64((uint64_t*)d_count, 0, 1, s));
  if (g->m <= 0) return PG_OK;
  const int32_t cap = (std::max(1, g->oriented->max_degree) + 1) & ~1;  // even: 8-byte aligned wave slices
  const size_t shmem = sizeof(int32_t) * ((size_t)kRowInts + (size_t)(sk ? 3 : 2) * cap) * kWaves;
  if (shmem > (size_t)kMaxLdsBytes)
    return fail(PG_E_UNSUPPORTED, sk ? "4-cliques: the largest oriented degree exceeds the on-chip C3 buffer (2720 with filters)"
                                     : "4-cliques: the largest oriented degree exceeds the on-chip C3 buffer (4080)");
  CliqueFilters f{};
  if (sk) {
    f.words = sk->words;
    f.ha = sk->ha;
    f.hc = sk->hc;
    f.B = sk->size;
    f.W = sk->W;
    f.b = sk->b;
  }
  const int64_t waves_needed = g->m;
  const unsigned grid = (unsigned)std::max<int64_t>(
      1, std::min<int64_t>((waves_needed + kWaves - 1) / kWaves, (int64_t)std::max(1, g->ctx->num_cus) * 8));
  ProfScope ps(s, sk ? "four_cliques_bf" : "four_cliques_exact");
#define PG_CK(WW)                                                                                                  \
  hipLaunchKernelGGL(k_four_cliques<WW>, dim3(grid), dim3(kBlock), shmem, s, g->poff, g->padj, g->parc_src, g->m, \
                     g->deg, cap, f, d_count)
  if (!sk) {
    PG_CK(-1);
  } else {
    switch (sk->W) {
      case 1: PG_CK(1); break;
      case 2: PG_CK(2); break;
      case 3: PG_CK(3); break;
      case 4: PG_CK(4); break;
      case 5: PG_CK(5); break;
      case 6: PG_CK(6); break;
      case 7: PG_CK(7); break;
      case 8: PG_CK(8); break;
      case 9: PG_CK(9); break;
      case 10: PG_CK(10); break;
      case 11: PG_CK(11); break;
      case 12: PG_CK(12); break;
      case 13: PG_CK(13); break;
      case 14: PG_CK(14); break;
      case 15: PG_CK(15); break;
      case 16: PG_CK(16); break;
      default: PG_CK(0); break;  // rows wider than 16 words are dense
    }
  }
#undef PG_CK
  PG_LAUNCH_CHECK();
  return PG_OK;
}

}  // namespace pg
