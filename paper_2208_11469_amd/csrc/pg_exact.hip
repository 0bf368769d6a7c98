// Exact intersection baselines on the same graphs: |N_u cap N_v| from the
// sorted neighbour lists (Fig. 1; the exact rows of Table "tab:queries-int"),
// the node-iterator triangle count over the degree orientation (Listing
// "lst:tc"), exact local clustering coefficients and Jaccard similarities.
//
// Intersection kernel: a wave takes 64 pairs. The elements of the shorter list
// of every pair become the wave's work items; they are spread evenly over the
// 64 lanes regardless of which pair they belong to, and each item is
// binary-searched in the longer list. This balances skewed degree mixes inside
// a wave, and the cost per pair is min(d_u, d_v) * log max(d_u, d_v).
//
// Bitmap variant (PG_EXACT_BITMAP): a block marks the list of one vertex v in
// an LDS bitmap of 2^20 IDs and every wave probes the list of one of v's
// neighbours against it, counting hits with ballots; then the block clears the
// bits it set. IDs beyond 2^20 are handled window by window. Cost per pair:
// d_u probes, no search.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pg_device.h"
#include "pg_internal.h"
#include "pg_pair.h"

namespace pg {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

__device__ __forceinline__ bool contains(const int32_t* __restrict__ a, int64_t lo, int64_t hi, int32_t key) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    const int32_t x = a[mid];
    if (x == key) return true;
    if (x < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return false;
}

struct WaveShared {
  int64_t excl[kWave];
  int64_t abeg[kWave];
  int64_t bbeg[kWave];
  int64_t blen[kWave];
  uint32_t cnt[kWave];
};

// Intersect the lane's pair of lists (a = shorter, b = longer, both in `lists`)
// cooperatively with the other lanes of the wave; returns the lane's count.
__device__ uint32_t wave_intersect(const int32_t* __restrict__ lists, int64_t abeg, int64_t alen, int64_t bbeg,
                                   int64_t blen, WaveShared& sh) {
  const int lane = lane_id();
  const int64_t work = (blen > 0) ? alen : 0;
  int64_t incl = work;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int64_t y = __shfl_up(incl, d);
    if (lane >= d) incl += y;
  }
  const int64_t total = __shfl(incl, kWave - 1);
  sh.excl[lane] = incl - work;
  sh.abeg[lane] = abeg;
  sh.bbeg[lane] = bbeg;
  sh.blen[lane] = blen;
  sh.cnt[lane] = 0;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int64_t t = lane; t < total; t += kWave) {
    // owner: the last lane q with excl[q] <= t
    int lo = 0, hi = kWave;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (sh.excl[mid] <= t)
        lo = mid;
      else
        hi = mid;
    }
    const int q = lo;
    const int32_t x = lists[sh.abeg[q] + (t - sh.excl[q])];
    if (contains(lists, sh.bbeg[q], sh.bbeg[q] + sh.blen[q], x)) atomicAdd(&sh.cnt[q], 1u);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const uint32_t r = sh.cnt[lane];
  __builtin_amdgcn_wave_barrier();
  return r;
}

// out[e] = |N_u cap N_v|; optional integer scatter of the count to both
// endpoints' sums (order-independent, so deterministic).
__global__ __launch_bounds__(kBlock) void k_exact_pairs(const int32_t* __restrict__ off,
                                                        const int32_t* __restrict__ adj, int32_t n,
                                                        const int32_t* __restrict__ pu, const int32_t* __restrict__ pv,
                                                        int64_t npairs, uint32_t* __restrict__ out,
                                                        unsigned long long* __restrict__ vsum) {
  __shared__ WaveShared shw[kWavesPerBlock];
  WaveShared& sh = shw[threadIdx.x / kWave];
  const int64_t nwaves_total = (int64_t)gridDim.x * kWavesPerBlock;
  for (int64_t wbase = (blockIdx.x * (int64_t)kWavesPerBlock + threadIdx.x / kWave) * kWave; wbase < npairs;
       wbase += nwaves_total * kWave) {
    const int64_t e = wbase + lane_id();
    int64_t abeg = 0, alen = 0, bbeg = 0, blen = 0;
    int32_t u = -1, v = -1;
    bool ok = false;
    if (e < npairs) {
      u = pu[e];
      v = pv[e];
      ok = (uint32_t)u < (uint32_t)n && (uint32_t)v < (uint32_t)n;
      if (ok) {
        const int64_t ub = off[u], ul = off[u + 1] - ub;
        const int64_t vb = off[v], vl = off[v + 1] - vb;
        if (ul <= vl) {
          abeg = ub; alen = ul; bbeg = vb; blen = vl;
        } else {
          abeg = vb; alen = vl; bbeg = ub; blen = ul;
        }
      }
    }
    const uint32_t c = wave_intersect(adj, abeg, alen, bbeg, blen, sh);
    if (e < npairs) {
      if (out) out[e] = ok ? c : 0xFFFFFFFFu;
      if (vsum && ok && c) {
        atomicAdd(&vsum[u], (unsigned long long)c);
        atomicAdd(&vsum[v], (unsigned long long)c);
      }
    }
  }
}

// Node iterator over the orientation: sum over oriented edges (v, u) of
// |N+_v cap N+_u|; one integer atomic per wave.
__global__ __launch_bounds__(kBlock) void k_exact_tc(const int32_t* __restrict__ poff, const int32_t* __restrict__ padj,
                                                     const int32_t* __restrict__ psrc, int64_t m,
                                                     unsigned long long* __restrict__ tc) {
  __shared__ WaveShared shw[kWavesPerBlock];
  WaveShared& sh = shw[threadIdx.x / kWave];
  const int64_t nwaves_total = (int64_t)gridDim.x * kWavesPerBlock;
  unsigned long long acc = 0;
  for (int64_t wbase = (blockIdx.x * (int64_t)kWavesPerBlock + threadIdx.x / kWave) * kWave; wbase < m;
       wbase += nwaves_total * kWave) {
    const int64_t p = wbase + lane_id();
    int64_t abeg = 0, alen = 0, bbeg = 0, blen = 0;
    if (p < m) {
      const int32_t v = psrc[p], u = padj[p];
      const int64_t vb = poff[v], vl = poff[v + 1] - vb;
      const int64_t ub = poff[u], ul = poff[u + 1] - ub;
      if (vl <= ul) {
        abeg = vb; alen = vl; bbeg = ub; blen = ul;
      } else {
        abeg = ub; alen = ul; bbeg = vb; blen = vl;
      }
    }
    acc += wave_intersect(padj, abeg, alen, bbeg, blen, sh);
  }
#pragma unroll
  for (int s = kWave / 2; s >= 1; s >>= 1) acc += __shfl_xor(acc, s);
  if (lane_id() == 0 && acc) atomicAdd(tc, acc);
}

__global__ void k_exact_cc_finish(const unsigned long long* __restrict__ vsum, const int32_t* __restrict__ deg,
                                  int32_t n, float* __restrict__ cc) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t d = deg[v];
  cc[v] = d >= 2 ? (float)((double)vsum[v] / ((double)d * ((double)d - 1.0))) : 0.0f;
}

// Similarity (Listing "lst:sim") of each pair from its exact intersection.
__global__ void k_exact_sim(const uint32_t* __restrict__ inter, const int32_t* __restrict__ deg, int32_t n,
                            const int32_t* __restrict__ pu, const int32_t* __restrict__ pv, int64_t npairs,
                            int measure, float* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < npairs; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = pu[e], v = pv[e];
    if ((uint32_t)u >= (uint32_t)n || (uint32_t)v >= (uint32_t)n) {
      out[e] = __int_as_float(0x7FC00000);
      continue;
    }
    out[e] = (float)similarity_of(measure, (double)inter[e], deg[u], deg[v]);
  }
}

// Jarvis-Patrick selection (Listing "lst:cl") of the m upper edges from their
// exact intersections: keep[e] = (similarity > tau) in FP64; |C| by integer
// atomics, one per block.
__global__ __launch_bounds__(kBlock) void k_exact_jp(const uint32_t* __restrict__ inter,
                                                     const int32_t* __restrict__ deg,
                                                     const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                                                     int64_t m, int measure, double tau, uint8_t* __restrict__ keep,
                                                     unsigned long long* __restrict__ kept) {
  __shared__ uint32_t block_kept;
  if (threadIdx.x == 0) block_kept = 0;
  __syncthreads();
  uint32_t mine = 0;
  for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < m; e += (int64_t)gridDim.x * kBlock) {
    const bool in = similarity_of(measure, (double)inter[e], deg[eu[e]], deg[ev[e]]) > tau;
    if (keep) keep[e] = in ? 1 : 0;
    mine += in ? 1u : 0u;
  }
  if (mine) atomicAdd(&block_kept, mine);
  __syncthreads();
  if (threadIdx.x == 0 && block_kept) atomicAdd(kept, (unsigned long long)block_kept);
}

constexpr int kBmBlock = 1024;
constexpr int kBmWaves = kBmBlock / kWave;
constexpr int kWinShift = 20;                    // IDs per window: 2^20 (a 128 KB bitmap)
constexpr int kWinWords = (1 << kWinShift) / 32;

// First position in a[lo, hi) with a[p] >= key.
__device__ __forceinline__ int64_t lower_bound_id(const int32_t* __restrict__ a, int64_t lo, int64_t hi, int64_t key) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)a[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// TC = false: for every vertex v, the counts |N_u cap N_v| of its upper
// neighbours u go to out[upoff[v] + j] (marked list N_v, probe lists N_u).
// TC = true: lists are the degree-oriented N+ (moff/madj); the counts of all
// oriented edges are summed into *tc. Blocks take vertices v = block, block +
// grid, ...; the bitmap starts clear and every pass clears what it set.
template <bool TC>
__global__ __launch_bounds__(kBmBlock) void k_exact_bitmap(const int32_t* __restrict__ moff,
                                                           const int32_t* __restrict__ madj,
                                                           const int32_t* __restrict__ ustart,
                                                           const int64_t* __restrict__ upoff, int32_t n,
                                                           uint32_t* __restrict__ out,
                                                           unsigned long long* __restrict__ tc) {
  extern __shared__ uint32_t bm[];
  for (int i = threadIdx.x; i < kWinWords; i += kBmBlock) bm[i] = 0;
  __syncthreads();
  const int w = threadIdx.x / kWave;
  const int lane = lane_id();
  unsigned long long acc = 0;
  for (int64_t v = blockIdx.x; v < n; v += gridDim.x) {
    const int64_t lb = moff[v], le = moff[v + 1];                  // marked list
    const int64_t pb = TC ? lb : (int64_t)ustart[v], pe = le;       // its neighbours to probe
    if (lb == le || pb == pe) continue;                             // uniform over the block
    const int64_t w_first = (int64_t)madj[lb] >> kWinShift, w_last = (int64_t)madj[le - 1] >> kWinShift;
    int64_t mlo = lb;
    for (int64_t win = w_first; win <= w_last; ++win) {
      const int64_t base = win << kWinShift;
      const int64_t mhi = lower_bound_id(madj, mlo, le, base + (1 << kWinShift));
      if (mhi == mlo) continue;  // no element of v's list in this window (uniform)
      for (int64_t q = mlo + threadIdx.x; q < mhi; q += kBmBlock) {
        const int32_t x = (int32_t)(madj[q] - base);
        atomicOr(&bm[x >> 5], 1u << (x & 31));
      }
      __syncthreads();
      for (int64_t j = pb + w; j < pe; j += kBmWaves) {  // one wave per neighbour u
        const int32_t u = madj[j];
        const int64_t ub = moff[u], ue = moff[u + 1];
        // one window holds every ID when n <= 2^20: the whole list, no search
        const bool whole = n <= (1 << kWinShift);
        const int64_t a = (whole || win == 0) ? ub : lower_bound_id(madj, ub, ue, base);
        const int64_t b = whole ? ue : lower_bound_id(madj, a, ue, base + (1 << kWinShift));
        uint32_t c = 0;
        for (int64_t q = a + lane; q < b + (kWave - 1) - ((b - a + kWave - 1) % kWave); q += kWave) {
          bool hit = false;
          if (q < b) {
            const int32_t x = (int32_t)(madj[q] - base);
            hit = (bm[x >> 5] >> (x & 31)) & 1u;
          }
          c += (uint32_t)__popcll(__ballot(hit));
        }
        if (lane == 0) {
          if constexpr (TC) {
            acc += c;
          } else {
            uint32_t* o = out + upoff[v] + (j - pb);
            *o = win == w_first ? c : *o + c;
          }
        }
      }
      __syncthreads();
      for (int64_t q = mlo + threadIdx.x; q < mhi; q += kBmBlock) bm[(madj[q] - base) >> 5] = 0;
      __syncthreads();
      mlo = mhi;
    }
  }
  if constexpr (TC) {
    if (lane == 0 && acc) atomicAdd(tc, acc);
  }
}

}  // namespace

int exact_pairs(const pg_graph* g, int algo, const int32_t* u, const int32_t* v, int64_t npairs, uint32_t* out,
                hipStream_t s) {
  if (algo == PG_EXACT_BITMAP) {
    // resolve_pairs turns u = v = NULL into the graph's own upper-edge lists
    if (u != g->eu || v != g->ev)
      return fail(PG_E_UNSUPPORTED, "PG_EXACT_BITMAP needs u = v = NULL (the m upper edges)");
    if (g->m <= 0 || g->n <= 0) return PG_OK;
    const unsigned grid = (unsigned)std::max(1, std::min(g->ctx->num_cus, g->n));
    ProfScope ps(s, "exact_bitmap");
    hipLaunchKernelGGL((k_exact_bitmap<false>), dim3(grid), dim3(kBmBlock), sizeof(uint32_t) * kWinWords, s, g->off,
                       g->adj, g->ustart, g->upoff, g->n, out, (unsigned long long*)nullptr);
    PG_LAUNCH_CHECK();
    return PG_OK;
  }
  if (algo != PG_EXACT_MERGE) return fail(PG_E_INVALID, "unknown exact algorithm");
  if (npairs <= 0) return PG_OK;
  const unsigned grid = grid_for((npairs + kWave - 1) / kWave * kWave, kBlock, 65536);
  ProfScope ps(s, "exact_pairs");
  hipLaunchKernelGGL(k_exact_pairs, dim3(grid), dim3(kBlock), 0, s, g->off, g->adj, g->n, u, v, npairs, out,
                     (unsigned long long*)nullptr);
  PG_LAUNCH_CHECK();
  return PG_OK;
}

int exact_tc(pg_graph* g, int algo, uint64_t* d_tc, hipStream_t s) {
  if (algo != PG_EXACT_MERGE && algo != PG_EXACT_BITMAP) return fail(PG_E_INVALID, "unknown exact algorithm");
  PG_TRY(graph_orient(g, s));
  PG_TRY(fill_u64(d_tc, 0, 1, s));
  if (g->m <= 0) return PG_OK;
  if (algo == PG_EXACT_BITMAP) {
    const unsigned grid = (unsigned)std::max(1, std::min(g->ctx->num_cus, g->n));
    ProfScope ps(s, "exact_tc_bitmap");
    hipLaunchKernelGGL((k_exact_bitmap<true>), dim3(grid), dim3(kBmBlock), sizeof(uint32_t) * kWinWords, s, g->poff,
                       g->padj, (const int32_t*)nullptr, (const int64_t*)nullptr, g->n, (uint32_t*)nullptr,
                       (unsigned long long*)d_tc);
    PG_LAUNCH_CHECK();
    return PG_OK;
  }
  const unsigned grid = grid_for((g->m + kWave - 1) / kWave * kWave, kBlock, 65536);
  ProfScope ps(s, "exact_tc");
  hipLaunchKernelGGL(k_exact_tc, dim3(grid), dim3(kBlock), 0, s, g->poff, g->padj, g->parc_src, g->m,
                     (unsigned long long*)d_tc);
  PG_LAUNCH_CHECK();
  return PG_OK;
}

int exact_cc(pg_graph* g, float* cc, hipStream_t s) {
  if (g->n <= 0) return PG_OK;
  uint64_t* vsum = nullptr;
  PG_TRY(dmalloc((void**)&vsum, sizeof(uint64_t) * (size_t)g->n, s));
  PG_TRY(fill_u64(vsum, 0, g->n, s));
  ProfScope ps(s, "exact_cc");
  if (g->m > 0) {
    const unsigned grid = grid_for((g->m + kWave - 1) / kWave * kWave, kBlock, 65536);
    hipLaunchKernelGGL(k_exact_pairs, dim3(grid), dim3(kBlock), 0, s, g->off, g->adj, g->n, g->eu, g->ev, g->m,
                       (uint32_t*)nullptr, (unsigned long long*)vsum);
    PG_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_exact_cc_finish, dim3(grid_for(g->n, kBlock, INT32_MAX)), dim3(kBlock), 0, s,
                     (const unsigned long long*)vsum, g->deg, g->n, cc);
  PG_LAUNCH_CHECK();
  return dfree(vsum, s);
}

int exact_similarity(const pg_graph* g, int measure, const int32_t* u, const int32_t* v, int64_t npairs, float* out,
                     hipStream_t s) {
  if (measure < PG_SIM_COMMON || measure > PG_SIM_TOTAL) return fail(PG_E_INVALID, "unknown similarity measure");
  if (npairs <= 0) return PG_OK;
  uint32_t* inter = nullptr;
  PG_TRY(dmalloc((void**)&inter, sizeof(uint32_t) * (size_t)npairs, s));
  int rc = exact_pairs(g, PG_EXACT_MERGE, u, v, npairs, inter, s);
  if (rc == PG_OK) {
    hipLaunchKernelGGL(k_exact_sim, dim3(grid_for(npairs, kBlock, 65536)), dim3(kBlock), 0, s, inter, g->deg, g->n,
                       u, v, npairs, measure, out);
    if (hipGetLastError() != hipSuccess) rc = fail(PG_E_DEVICE, "k_exact_sim launch failed");
  }
  dfree(inter, s);
  return rc;
}

int exact_jp(const pg_graph* g, int algo, int measure, double tau, uint8_t* keep, unsigned long long* d_kept,
             hipStream_t s) {
  if (measure < PG_SIM_COMMON || measure > PG_SIM_TOTAL) return fail(PG_E_INVALID, "unknown similarity measure");
  if (algo != PG_EXACT_MERGE && algo != PG_EXACT_BITMAP) return fail(PG_E_INVALID, "unknown exact algorithm");
  PG_TRY(fill_u64((uint64_t*)d_kept, 0, 1, s));
  if (g->m <= 0) return PG_OK;
  uint32_t* inter = nullptr;
  PG_TRY(dmalloc((void**)&inter, sizeof(uint32_t) * (size_t)g->m, s));
  int rc = exact_pairs(g, algo, g->eu, g->ev, g->m, inter, s);
  if (rc == PG_OK) {
    ProfScope ps(s, "exact_jarvis_patrick");
    // a few blocks per CU: each block adds its count to one shared counter
    const unsigned grid = grid_for(g->m, kBlock, (int64_t)std::max(1, g->ctx->num_cus) * 8);
    hipLaunchKernelGGL(k_exact_jp, dim3(grid), dim3(kBlock), 0, s, inter, g->deg, g->eu,
                       g->ev, g->m, measure, tau, keep, d_kept);
    if (hipGetLastError() != hipSuccess) rc = fail(PG_E_DEVICE, "k_exact_jp launch failed");
  }
  dfree(inter, s);
  return rc;
}

}  // namespace pg
