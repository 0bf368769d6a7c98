// Graph ingest on the device: CSR checks, degrees, the degree-bin partition of
// the vertices, the m undirected edges (v, u), v < u, in CSR order, arc
// sources, and the degree orientation used by the exact node iterator
// (Listing "lst:tc"). Also the scan / fill / fixed-order sum utilities.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <new>
#include <vector>

#include "pg_device.h"
#include "pg_internal.h"

namespace pg {
namespace {

constexpr int kBlock = 256;

// Error bits raised by the checks.
constexpr int kBadOffsets = 1, kBadRange = 2, kSelfLoop = 4, kUnsorted = 8, kAsymmetric = 16;

__global__ void k_check_offsets(const int32_t* __restrict__ off, int32_t n, int64_t nnz, int* flags) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v > n) return;
  bool bad = false;
  if (v == 0 && off[0] != 0) bad = true;
  if (v == n && (int64_t)off[n] != nnz) bad = true;
  if (v < n && off[v + 1] < off[v]) bad = true;
  if (v <= n && (off[v] < 0 || (int64_t)off[v] > nnz)) bad = true;
  if (bad) atomicOr(flags, kBadOffsets);
}

__global__ void k_check_range(const int32_t* __restrict__ adj, int64_t nnz, int32_t n, int* flags) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = adj[p];
    if (x < 0 || x >= n) atomicOr(flags, kBadRange);
  }
}

// Lower bound of key in a[lo, hi) (a sorted ascending).
__device__ __forceinline__ int64_t lower_bound_i32(const int32_t* __restrict__ a, int64_t lo, int64_t hi, int32_t key) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Source vertex of arc p: the last v with off[v] <= p (offsets validated).
__device__ __forceinline__ int32_t arc_source(const int32_t* __restrict__ off, int32_t n, int64_t p) {
  int32_t lo = 0, hi = n;  // answer in [0, n)
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if ((int64_t)off[mid] <= p)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Sortedness, duplicates, self-loops and symmetry (u in N_v => v in N_u).
__global__ void k_check_structure(const int32_t* __restrict__ off, const int32_t* __restrict__ adj, int32_t n,
                                  int64_t nnz, int* flags) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = arc_source(off, n, p);
    const int32_t u = adj[p];
    int f = 0;
    if (u == v) f |= kSelfLoop;
    if (p > off[v] && adj[p - 1] >= u) f |= kUnsorted;
    const int64_t q = lower_bound_i32(adj, off[u], off[u + 1], v);
    if (q >= off[u + 1] || adj[q] != v) f |= kAsymmetric;
    if (f) atomicOr(flags, f);
  }
}

__global__ void k_degrees(const int32_t* __restrict__ off, int32_t n, int32_t* __restrict__ deg, int* max_deg,
                          unsigned long long* wedges) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int32_t d = 0;
  if (v < n) {
    d = off[v + 1] - off[v];
    deg[v] = d;
  }
  // wave-level combine, one atomic per wave (integer: order-independent)
  unsigned long long w = (unsigned long long)d * (unsigned long long)(d > 0 ? d - 1 : 0) / 2ull;
  int mx = d;
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) {
    w += __shfl_xor(w, s);
    const int o = __shfl_xor(mx, s);
    mx = o > mx ? o : mx;
  }
  if (lane_id() == 0) {
    atomicMax(max_deg, mx);
    atomicAdd(wedges, w);
  }
}

__device__ __forceinline__ int degree_bin(int32_t d) {
  return d <= kBinMaxDeg[0] ? 0 : d <= kBinMaxDeg[1] ? 1 : d <= kBinMaxDeg[2] ? 2 : 3;
}

__global__ void k_degree_bin_keys(const int32_t* __restrict__ deg, int32_t n, uint8_t* __restrict__ key) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v < n) key[v] = (uint8_t)degree_bin(deg[v]);
}

// Plan tier of a count of arcs: 1 light, 2 medium, 3 heavy.
__device__ __forceinline__ uint8_t plan_tier(int64_t d, int64_t light_max = kLightMax) {
  return d <= light_max ? 1 : (d <= kMediumMax ? 2 : 3);
}

// Vertices without arcs, added into *count (one atomic per wave).
__global__ void k_count_empty(const int32_t* __restrict__ off, int32_t n, unsigned long long* __restrict__ count) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const uint64_t ball = __ballot(v < n && off[v + 1] == off[v]);
  if (lane_id() == 0 && ball) atomicAdd(count, (unsigned long long)__popcll(ball));
}

__global__ void k_plan_keys(const int32_t* __restrict__ off, int32_t n, uint8_t* __restrict__ key) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v < n) key[v] = plan_tier(off[v + 1] - off[v]);
}

// Slab-plan keys. Items (x, v), x < kSlabs, at key[x*n + v]: the tier of v's
// upper neighbours in slab x, 0 when there are none or v is not sliced. Whole
// vertices at key[kSlabs*n + v]: 1 for a whole vertex, else 0.
__global__ void k_slab_keys(const int32_t* __restrict__ off, const int32_t* __restrict__ ustart,
                            const int32_t* __restrict__ split, int32_t n, uint8_t* __restrict__ key) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)(kSlabs + 1) * n) return;
  const int x = (int)(i / n);
  const int32_t v = (int32_t)(i % n);
  const int32_t dup = off[v + 1] - ustart[v];
  if (x == kSlabs) {
    key[i] = (dup >= 1 && dup <= kSliceMin) ? 1 : 0;
    return;
  }
  const int64_t d = slab_end(off, split, (size_t)n, x, v) - slab_begin(ustart, split, (size_t)n, x, v);
  key[i] = (dup <= kSliceMin || d == 0) ? 0 : plan_tier(d, kSlabLightMax);
}

// Stable partition of the vertices by a small key (< kNumBins): per-block
// counts, key-major.
__global__ void k_part_count(const uint8_t* __restrict__ keys, int32_t n, int64_t* __restrict__ counts, int64_t nblk) {
  __shared__ int wc[kBlock / kWave][kNumBins];
  const int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  const int key = v < n ? (int)keys[v] : -1;
  const int w = threadIdx.x / kWave;
#pragma unroll
  for (int j = 0; j < kNumBins; ++j) {
    const unsigned long long bal = __ballot(key == j);
    if (lane_id() == 0) wc[w][j] = __popcll(bal);
  }
  __syncthreads();
  if (threadIdx.x < kNumBins) {
    int64_t t = 0;
    for (int i = 0; i < kBlock / kWave; ++i) t += wc[i][threadIdx.x];
    counts[threadIdx.x * nblk + blockIdx.x] = t;
  }
}

__global__ void k_part_scatter(const uint8_t* __restrict__ keys, int32_t n, const int64_t* __restrict__ base,
                               int64_t nblk, int32_t* __restrict__ out) {
  __shared__ int wc[kBlock / kWave][kNumBins];
  const int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  const int key = v < n ? (int)keys[v] : -1;
  const int w = threadIdx.x / kWave;
  unsigned long long mine = 0;
#pragma unroll
  for (int j = 0; j < kNumBins; ++j) {
    const unsigned long long bal = __ballot(key == j);
    if (lane_id() == 0) wc[w][j] = __popcll(bal);
    if (key == j) mine = bal;
  }
  __syncthreads();
  if (key >= 0) {
    int64_t rank = __popcll(mine & ((1ull << lane_id()) - 1ull));
    for (int i = 0; i < w; ++i) rank += wc[i][key];
    out[base[key * nblk + blockIdx.x] + rank] = (int32_t)v;
  }
}

// Arc ranges of listed vertices: over N_v (x < 0) or of item (x, v).
__global__ void k_heavy_ranges(const int32_t* __restrict__ verts, int64_t count, const int32_t* __restrict__ off,
                               const int32_t* __restrict__ ustart, const int32_t* __restrict__ split, int32_t n, int x,
                               int64_t* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int32_t v = verts[i];
  out[2 * i] = x < 0 ? off[v] : slab_begin(ustart, split, (size_t)n, x, v);
  out[2 * i + 1] = x < 0 ? off[v + 1] : slab_end(off, split, (size_t)n, x, v);
}

// ---- per-vertex group kernels: G lanes per vertex, G <= 256 divides 256 -----

// Number of neighbours above v (the suffix of the sorted N_v).
template <int G>
__global__ void k_upper_count(const int32_t* __restrict__ off, const int32_t* __restrict__ adj,
                              const int32_t* __restrict__ verts, int64_t nverts, int64_t* __restrict__ cnt,
                              int32_t* __restrict__ ustart) {
  const int64_t grp = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x % G;
  if (grp >= nverts || lane != 0) return;
  const int32_t v = verts[grp];
  const int64_t fg = lower_bound_i32(adj, off[v], off[v + 1], v + 1);
  cnt[v] = off[v + 1] - fg;
  ustart[v] = (int32_t)fg;
}

template <int G>
__global__ void k_upper_fill(const int32_t* __restrict__ off, const int32_t* __restrict__ adj,
                             const int32_t* __restrict__ verts, int64_t nverts, const int64_t* __restrict__ up_off,
                             int32_t* __restrict__ eu, int32_t* __restrict__ ev) {
  const int64_t grp = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x % G;
  if (grp >= nverts) return;
  const int32_t v = verts[grp];
  const int64_t end = off[v + 1];
  const int64_t cnt = up_off[v + 1] - up_off[v];
  const int64_t fg = end - cnt;
  const int64_t e0 = up_off[v];
  for (int64_t j = fg + lane; j < end; j += G) {
    eu[e0 + (j - fg)] = v;
    ev[e0 + (j - fg)] = adj[j];
  }
}

template <int G>
__global__ void k_arc_src(const int32_t* __restrict__ off, const int32_t* __restrict__ verts, int64_t nverts,
                          int32_t* __restrict__ src) {
  const int64_t grp = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x % G;
  if (grp >= nverts) return;
  const int32_t v = verts[grp];
  for (int64_t p = off[v] + lane; p < off[v + 1]; p += G) src[p] = v;
}

// Degree order R: R(v) < R(u) iff (d_v, v) < (d_u, u) (Listing "lst:tc").
__device__ __forceinline__ bool rank_less(const int32_t* __restrict__ deg, int32_t v, int32_t u) {
  const int32_t dv = deg[v], du = deg[u];
  return dv < du || (dv == du && v < u);
}

template <int G>
__global__ void k_orient_count(const int32_t* __restrict__ off, const int32_t* __restrict__ adj,
                               const int32_t* __restrict__ deg, const int32_t* __restrict__ verts, int64_t nverts,
                               int64_t* __restrict__ cnt) {
  __shared__ int64_t part[kBlock];
  const int64_t grp = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x % G;
  int64_t c = 0;
  int32_t v = -1;
  if (grp < nverts) {
    v = verts[grp];
    for (int64_t p = off[v] + lane; p < off[v + 1]; p += G) c += rank_less(deg, v, adj[p]) ? 1 : 0;
  }
  part[threadIdx.x] = c;
  __syncthreads();
  if (grp < nverts && lane == 0) {
    int64_t t = 0;
    for (int i = 0; i < G; ++i) t += part[threadIdx.x + i];
    cnt[v] = t;
  }
}

// Keeps the order of N_v, so every N+_v stays sorted by ID. G <= 64 lanes per
// vertex, so a group never straddles a wave; output positions come from a
// ballot prefix inside the group.
template <int G>
__global__ void k_orient_fill(const int32_t* __restrict__ off, const int32_t* __restrict__ adj,
                              const int32_t* __restrict__ deg, const int32_t* __restrict__ verts, int64_t nverts,
                              const int64_t* __restrict__ poff, int32_t* __restrict__ padj, int32_t* __restrict__ psrc) {
  static_assert(G <= kWave, "group must fit in a wave");
  const int64_t grp = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x % G;
  if (grp >= nverts) return;
  const int32_t v = verts[grp];
  const int64_t end = off[v + 1];
  int64_t q = poff[v];
  const int shift = lane_id() - lane;  // first lane of this group inside the wave
  const unsigned long long gmask = G == 64 ? ~0ull : ((1ull << G) - 1ull);
  for (int64_t p0 = off[v]; p0 < end; p0 += G) {
    const int64_t p = p0 + lane;
    const bool keep = (p < end) && rank_less(deg, v, adj[p]);
    const unsigned long long bits = (__ballot(keep) >> shift) & gmask;
    if (keep) {
      const int before = __popcll(bits & ((1ull << lane) - 1ull));
      padj[q + before] = adj[p];
      psrc[q + before] = v;
    }
    q += __popcll(bits);
  }
}

// ---- scan ------------------------------------------------------------------

constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__device__ __forceinline__ int64_t wave_incl_scan(int64_t x) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int64_t y = __shfl_up(x, d);
    if (lane_id() >= d) x += y;
  }
  return x;
}

__global__ void k_scan_tile(const int64_t* __restrict__ in, int64_t* __restrict__ out, int64_t count,
                            int64_t* __restrict__ tile_sums) {
  __shared__ int64_t wsum[kBlock / kWave];
  const int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * (int64_t)kScanItems;
  int64_t v[kScanItems];
  int64_t sum = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + i;
    v[i] = idx < count ? in[idx] : 0;
    sum += v[i];
  }
  const int64_t incl = wave_incl_scan(sum);
  const int w = threadIdx.x / kWave;
  if (lane_id() == kWave - 1) wsum[w] = incl;
  __syncthreads();
  int64_t wbase = 0, total = 0;
#pragma unroll
  for (int i = 0; i < kBlock / kWave; ++i) {
    wbase += (i < w) ? wsum[i] : 0;
    total += wsum[i];
  }
  int64_t run = wbase + incl - sum;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + i;
    if (idx < count) out[idx] = run;
    run += v[i];
  }
  if (threadIdx.x == 0 && tile_sums) tile_sums[blockIdx.x] = total;
}

__global__ void k_scan_add(int64_t* __restrict__ out, int64_t count, const int64_t* __restrict__ tile_off) {
  const int64_t base = blockIdx.x * (int64_t)kScanTile;
  const int64_t add = tile_off[blockIdx.x];
  for (int i = threadIdx.x; i < kScanTile; i += kBlock) {
    const int64_t idx = base + i;
    if (idx < count) out[idx] += add;
  }
}

// Incoming upper arcs from sliced vertices (those with more than kSliceMin
// upper neighbours): every upper arc (u, v) of a sliced u adds one to cnt[v].
// G lanes per vertex u; integer atomics, so the counts are exact.
template <int G>
__global__ void k_in_sliced(const int32_t* __restrict__ off, const int32_t* __restrict__ ustart,
                            const int32_t* __restrict__ adj, const int32_t* __restrict__ verts, int64_t nverts,
                            unsigned long long* __restrict__ cnt) {
  const int64_t grp = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x % G;
  if (grp >= nverts) return;
  const int32_t u = verts[grp];
  const int64_t beg = ustart[u], end = off[u + 1];
  if (end - beg <= kSliceMin) return;
  for (int64_t p = beg + lane; p < end; p += G) atomicAdd(&cnt[adj[p]], 1ull);
}

// Slab boundaries: lo[x] is the first vertex whose exclusive prefix of
// incoming sliced arcs reaches x/kSlabs of the total (lo[0] = 0, lo[kSlabs] = n).
__global__ void k_slab_bounds(const int64_t* __restrict__ pre, const int64_t* __restrict__ cnt, int32_t n,
                              int32_t* __restrict__ lo) {
  const int x = threadIdx.x;
  if (x > kSlabs) return;
  if (x == 0 || x == kSlabs) {
    lo[x] = x == 0 ? 0 : n;
    return;
  }
  const int64_t total = n > 0 ? pre[n - 1] + cnt[n - 1] : 0;
  const int64_t target = total * x / kSlabs;
  int64_t a = 0, b = n;  // first v in [0, n) with pre[v] >= target, n if none
  while (a < b) {
    const int64_t mid = (a + b) >> 1;
    if (pre[mid] < target)
      a = mid + 1;
    else
      b = mid;
  }
  lo[x] = (int32_t)a;
}

__global__ void k_slab_split(const int32_t* __restrict__ off, const int32_t* __restrict__ ustart,
                             const int32_t* __restrict__ adj, int32_t n, const int32_t* __restrict__ lo,
                             int32_t* __restrict__ split) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int64_t beg = ustart[v], end = off[v + 1];
    int64_t p = beg;
    for (int x = 1; x < kSlabs; ++x) {
      p = lower_bound_i32(adj, p, end, lo[x]);
      split[(size_t)(x - 1) * n + v] = (int32_t)p;
    }
  }
}

// Sort key of listed items: ceil(arcs / bucket), the arcs of (x, v) for slab
// x >= 0, else off[v+1] - ustart[v] (upper neighbours, or all of N_v when
// ustart = off), at most 255 (longer items share the first place).
__global__ void k_item_keys(const int32_t* __restrict__ verts, int64_t count, int x, int bucket,
                            const int32_t* __restrict__ off,
                            const int32_t* __restrict__ ustart, const int32_t* __restrict__ split, int32_t n,
                            uint8_t* __restrict__ key) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int32_t v = verts[i];
  const int64_t d = x < 0 ? off[v + 1] - ustart[v]
                          : slab_end(off, split, (size_t)n, x, v) - slab_begin(ustart, split, (size_t)n, x, v);
  key[i] = (uint8_t)std::min<int64_t>((d + bucket - 1) / bucket, 255);  // ceil(d / bucket): 0 only without arcs
}

// Sliced vertices (more than kSliceMin arcs in [begin[v], off[v+1])) as 0/1.
__global__ void k_sliced_flags(const int32_t* __restrict__ off, const int32_t* __restrict__ begin, int32_t n,
                               int64_t* __restrict__ flag) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v < n) flag[v] = off[v + 1] - begin[v] > kSliceMin ? 1 : 0;
}

// Rank of each sliced vertex among them (its exclusive prefix), -1 otherwise.
__global__ void k_sliced_rank(const int64_t* __restrict__ flag, const int64_t* __restrict__ pre, int32_t n,
                              int32_t* __restrict__ rank) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v < n) rank[v] = flag[v] ? (int32_t)pre[v] : -1;
}

// Complemented 2-bit digit `pass` of a key: partitioning by it, least
// significant digit first, sorts by descending key.
__global__ void k_desc_digit(const uint8_t* __restrict__ key, int64_t count, int pass, uint8_t* __restrict__ digit) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) digit[i] = (uint8_t)(3 - ((key[i] >> (2 * pass)) & 3));
}

__global__ void k_permute(const int32_t* __restrict__ perm, const int32_t* __restrict__ vals,
                          const uint8_t* __restrict__ key, int64_t count, int32_t* __restrict__ vals_out,
                          uint8_t* __restrict__ key_out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int32_t j = perm[i];
  vals_out[i] = vals[j];
  key_out[i] = key[j];
}

__global__ void k_fill_u64(uint64_t* __restrict__ p, uint64_t value, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

// Single block: thread t adds entries t, t + 256, ... in order; fixed tree.
__global__ void k_sum_chunks(const double* __restrict__ chunks, int64_t nchunks, double divisor, double* out) {
  __shared__ double lds[kBlock / kWave];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < nchunks; i += kBlock) acc += chunks[i];
  const double r = block_sum_256(acc, lds);
  if (threadIdx.x == 0) out[0] = r / divisor;
}

// One block of kWideBlock threads over up to kWideMax partials: thread t sums
// entries t, t + kWideBlock, ... in rounds of kWideLoads independent loads
// (zero past the end) into eight accumulators in a fixed pattern, then a
// fixed tree. One launch instead of two for the usual partial counts; the
// loads of a round are all in flight together.
constexpr int kWideBlock = 1024;
constexpr int kWideLoads = 16;
constexpr int64_t kWideMax = 1 << 17;

__global__ __launch_bounds__(kWideBlock) void k_sum_wide(const double* __restrict__ chunks, int64_t nchunks,
                                                         double divisor, double* out) {
  __shared__ double lds[kWideBlock / kWave];
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t i0 = threadIdx.x; i0 < nchunks; i0 += (int64_t)kWideLoads * kWideBlock) {
    double v[kWideLoads];
#pragma unroll
    for (int j = 0; j < kWideLoads; ++j) {
      const int64_t i = i0 + (int64_t)j * kWideBlock;
      v[j] = i < nchunks ? chunks[i] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kWideLoads; ++j) a[j & 7] += v[j];
  }
  double acc = group_sum<kWave>(((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7])));
  if (lane_id() == 0) lds[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < kWideBlock / kWave; ++w) r += lds[w];
    out[0] = r / divisor;
  }
}

// Partials of a plain array over fixed chunks of 2048 entries.
__global__ void k_array_chunks(const double* __restrict__ x, int64_t count, double* __restrict__ chunks) {
  __shared__ double lds[kBlock / kWave];
  const int64_t nchunks = (count + kScanTile - 1) / kScanTile;
  for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    double acc = 0.0;
    for (int j = 0; j < kScanItems; ++j) {
      const int64_t i = ch * kScanTile + (int64_t)j * kBlock + threadIdx.x;
      if (i < count) acc += x[i];
    }
    const double r = block_sum_256(acc, lds);
    if (threadIdx.x == 0) chunks[ch] = r;
  }
}

__global__ void k_i64_to_i32(const int64_t* __restrict__ in, int32_t* __restrict__ out, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (int32_t)in[i];
}

}  // namespace

// ---- host side ---------------------------------------------------------------

int exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t count, hipStream_t s) {
  if (count <= 0) return PG_OK;
  const int64_t ntiles = (count + kScanTile - 1) / kScanTile;
  if (ntiles == 1) {
    hipLaunchKernelGGL(k_scan_tile, dim3(1), dim3(kBlock), 0, s, in, out, count, (int64_t*)nullptr);
    PG_LAUNCH_CHECK();
    return PG_OK;
  }
  int64_t* sums = nullptr;
  PG_TRY(dmalloc((void**)&sums, sizeof(int64_t) * 2 * ntiles, s));
  int64_t* offs = sums + ntiles;
  hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)ntiles), dim3(kBlock), 0, s, in, out, count, sums);
  PG_LAUNCH_CHECK();
  PG_TRY(exclusive_scan_i64(sums, offs, ntiles, s));
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)ntiles), dim3(kBlock), 0, s, out, count, offs);
  PG_LAUNCH_CHECK();
  return dfree(sums, s);
}

int fill_u64(uint64_t* p, uint64_t value, int64_t count, hipStream_t s) {
  if (count <= 0) return PG_OK;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(count, kBlock, 4096)), dim3(kBlock), 0, s, p, value, count);
  PG_LAUNCH_CHECK();
  return PG_OK;
}

int64_t sum_chunks_tiles(int64_t nchunks) {
  return (nchunks > 4 * kScanTile && nchunks > kWideMax) ? (nchunks + kScanTile - 1) / kScanTile : 0;
}

int sum_chunks(const double* chunks, int64_t nchunks, double divisor, double* out, hipStream_t s, double* tiles) {
  ProfScope ps(s, "sum_chunks");
  if (nchunks > 4 * kScanTile && nchunks <= kWideMax) {
    hipLaunchKernelGGL(k_sum_wide, dim3(1), dim3(kWideBlock), 0, s, chunks, nchunks, divisor, out);
    PG_LAUNCH_CHECK();
    return PG_OK;
  }
  if (nchunks > 4 * kScanTile) {
    // two levels: fixed tiles of kScanTile partials, then the tile sums
    const int64_t nt = sum_chunks_tiles(nchunks);
    const bool own = tiles == nullptr;
    if (own) PG_TRY(dmalloc((void**)&tiles, sizeof(double) * nt, s));
    hipLaunchKernelGGL(k_array_chunks, dim3((unsigned)std::min<int64_t>(nt, 65536)), dim3(kBlock), 0, s, chunks,
                       nchunks, tiles);
    PG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sum_chunks, dim3(1), dim3(kBlock), 0, s, (const double*)tiles, nt, divisor, out);
    PG_LAUNCH_CHECK();
    return own ? dfree(tiles, s) : PG_OK;
  }
  hipLaunchKernelGGL(k_sum_chunks, dim3(1), dim3(kBlock), 0, s, chunks, nchunks, divisor, out);
  PG_LAUNCH_CHECK();
  return PG_OK;
}

int sum_array(const double* x, int64_t count, double divisor, double* out, hipStream_t s) {
  const int64_t nchunks = std::max<int64_t>(1, (count + kScanTile - 1) / kScanTile);
  double* chunks = nullptr;
  PG_TRY(dmalloc((void**)&chunks, sizeof(double) * nchunks, s));
  PG_TRY(fill_u64((uint64_t*)chunks, 0, nchunks, s));  // a kernel, not a memset node, under graph capture
  if (count > 0) {
    hipLaunchKernelGGL(k_array_chunks, dim3((unsigned)std::min<int64_t>(nchunks, 65536)), dim3(kBlock), 0, s, x, count,
                       chunks);
    PG_LAUNCH_CHECK();
  }
  PG_TRY(sum_chunks(chunks, nchunks, divisor, out, s));
  return dfree(chunks, s);
}

namespace {

// Launch a group-per-vertex kernel over every degree bin.
#define PG_FOR_BINS(KERNEL, g, s, ...)                                                               \
  do {                                                                                               \
    for (int bin_ = 0; bin_ < kNumBins; ++bin_) {                                                    \
      const int64_t cnt_ = (g)->bin_start[bin_ + 1] - (g)->bin_start[bin_];                          \
      if (cnt_ <= 0) continue;                                                                       \
      const int32_t* verts_ = (g)->bin_verts + (g)->bin_start[bin_];                                 \
      const int G_ = kBinGroup[bin_];                                                                \
      const unsigned grid_ = (unsigned)((cnt_ * G_ + kBlock - 1) / kBlock);                          \
      if (G_ == 4)                                                                                   \
        hipLaunchKernelGGL(KERNEL<4>, dim3(grid_), dim3(kBlock), 0, s, __VA_ARGS__);                 \
      else if (G_ == 16)                                                                             \
        hipLaunchKernelGGL(KERNEL<16>, dim3(grid_), dim3(kBlock), 0, s, __VA_ARGS__);                \
      else if (G_ == 64)                                                                             \
        hipLaunchKernelGGL(KERNEL<64>, dim3(grid_), dim3(kBlock), 0, s, __VA_ARGS__);                \
      else                                                                                           \
        hipLaunchKernelGGL(KERNEL<256>, dim3(grid_), dim3(kBlock), 0, s, __VA_ARGS__);               \
      PG_LAUNCH_CHECK();                                                                             \
    }                                                                                                \
  } while (0)

}  // namespace

namespace {

// Stable partition of the indices 0..n-1 into `out` by keys[i] < kNumBins.
// starts[j] is the first position of key j, starts[kNumBins] = n.
int partition_keys(const uint8_t* keys, int32_t n, int32_t* out, int64_t* starts, hipStream_t s) {
  for (int j = 0; j <= kNumBins; ++j) starts[j] = n <= 0 ? 0 : n;
  if (n <= 0) return PG_OK;
  const int64_t nblk = ((int64_t)n + kBlock - 1) / kBlock;
  int64_t* counts = nullptr;
  PG_TRY(dmalloc((void**)&counts, sizeof(int64_t) * 2 * kNumBins * nblk, s));
  int64_t* base = counts + kNumBins * nblk;
  hipLaunchKernelGGL(k_part_count, dim3((unsigned)nblk), dim3(kBlock), 0, s, keys, n, counts, nblk);
  PG_LAUNCH_CHECK();
  PG_TRY(exclusive_scan_i64(counts, base, kNumBins * nblk, s));
  hipLaunchKernelGGL(k_part_scatter, dim3((unsigned)nblk), dim3(kBlock), 0, s, keys, n, base, nblk, out);
  PG_LAUNCH_CHECK();
  for (int j = 0; j < kNumBins; ++j)
    PG_HIP(hipMemcpyAsync(&starts[j], base + j * nblk, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  PG_HIP(hipStreamSynchronize(s));
  starts[kNumBins] = n;
  return dfree(counts, s);
}

// Stable partition of all vertices by degree bin (by_plan false) or by plan
// tier over N_v (by_plan true).
int partition(pg_graph* g, bool by_plan, int32_t* out, int64_t* starts, hipStream_t s) {
  const int32_t n = g->n;
  if (n <= 0) return partition_keys(nullptr, 0, out, starts, s);
  const unsigned nblk = (unsigned)(((int64_t)n + kBlock - 1) / kBlock);
  uint8_t* keys = nullptr;
  PG_TRY(dmalloc((void**)&keys, (size_t)n, s));
  if (by_plan)
    hipLaunchKernelGGL(k_plan_keys, dim3(nblk), dim3(kBlock), 0, s, g->off, n, keys);
  else
    hipLaunchKernelGGL(k_degree_bin_keys, dim3(nblk), dim3(kBlock), 0, s, g->deg, n, keys);
  PG_LAUNCH_CHECK();
  PG_TRY(partition_keys(keys, n, out, starts, s));
  return dfree(keys, s);
}

// Stable sort of vals[0 .. count) by descending key[] (keys < 256): LSD radix
// with the 4-way partition, 2 bits per pass. vals and key are sorted in place.
int sort_desc_small(int32_t* vals, uint8_t* key, int64_t count, hipStream_t s) {
  if (count <= 1) return PG_OK;
  const unsigned grid = (unsigned)((count + kBlock - 1) / kBlock);
  uint8_t* digit = nullptr;
  int32_t* perm = nullptr;
  int32_t* vals2 = nullptr;
  uint8_t* key2 = nullptr;
  PG_TRY(dmalloc((void**)&perm, sizeof(int32_t) * 2 * (size_t)count + 2 * (size_t)count, s));
  vals2 = perm + count;
  digit = (uint8_t*)(vals2 + count);
  key2 = digit + count;
  int32_t* a = vals;
  uint8_t* ka = key;
  int32_t* b = vals2;
  uint8_t* kb = key2;
  for (int pass = 0; pass < 4; ++pass) {  // 4 passes: the result ends in the input buffers
    hipLaunchKernelGGL(k_desc_digit, dim3(grid), dim3(kBlock), 0, s, (const uint8_t*)ka, count, pass, digit);
    PG_LAUNCH_CHECK();
    int64_t starts[kNumBins + 1];
    PG_TRY(partition_keys(digit, (int32_t)count, perm, starts, s));
    hipLaunchKernelGGL(k_permute, dim3(grid), dim3(kBlock), 0, s, (const int32_t*)perm, (const int32_t*)a,
                       (const uint8_t*)ka, count, b, kb);
    PG_LAUNCH_CHECK();
    std::swap(a, b);
    std::swap(ka, kb);
  }
  return dfree(perm, s);
}

// Sorts a light list (slab x, or whole vertices for x < 0) by descending
// ceil(arcs / bucket), keeping ID order among equal keys (stable radix). With
// bucket = the arcs a group of the consuming kernel covers per pass, the
// groups of a wave take equally many passes while neighbouring groups keep
// nearby IDs, so their offsets, rows and outputs share cache lines. Items
// without arcs end the list.
int sort_light_list(int32_t* verts, int64_t count, int x, int bucket, pg_graph* g, const int32_t* off,
                    const int32_t* ustart, const int32_t* split, hipStream_t s) {
  if (count <= 1) return PG_OK;
  uint8_t* key = nullptr;
  PG_TRY(dmalloc((void**)&key, (size_t)count, s));
  hipLaunchKernelGGL(k_item_keys, dim3((unsigned)((count + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     (const int32_t*)verts, count, x, bucket, off, ustart, split, g->n, key);
  PG_LAUNCH_CHECK();
  PG_TRY(sort_desc_small(verts, key, count, s));
  return dfree(key, s);
}

// Heavy-tier chunks: the arc ranges of `nh` listed vertices (read back from
// the device) cut into pieces of at most kHeavyChunk arcs, appended to the
// host vectors. `slot` numbers the vertices from slot0.
int heavy_chunks(const int32_t* d_verts, int64_t nh, pg_graph* g, const int32_t* begin, const int32_t* split, int x,
                 int32_t slot0, std::vector<int32_t>& cv,
                 std::vector<int64_t>& cb, std::vector<int64_t>& ce, std::vector<int32_t>& cslot,
                 std::vector<int32_t>& first, hipStream_t s) {
  if (nh <= 0) return PG_OK;
  std::vector<int64_t> ranges(2 * (size_t)nh);
  std::vector<int32_t> hv((size_t)nh);
  int64_t* d_ranges = nullptr;
  PG_TRY(dmalloc((void**)&d_ranges, sizeof(int64_t) * 2 * nh, s));
  hipLaunchKernelGGL(k_heavy_ranges, dim3((unsigned)((nh + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, d_verts, nh,
                     g->off, begin, split, g->n, x, d_ranges);
  PG_LAUNCH_CHECK();
  PG_HIP(hipMemcpyAsync(ranges.data(), d_ranges, sizeof(int64_t) * 2 * nh, hipMemcpyDeviceToHost, s));
  PG_HIP(hipMemcpyAsync(hv.data(), d_verts, sizeof(int32_t) * nh, hipMemcpyDeviceToHost, s));
  PG_HIP(hipStreamSynchronize(s));
  PG_TRY(dfree(d_ranges, s));
  for (int64_t h = 0; h < nh; ++h) {
    first.push_back((int32_t)cv.size());
    for (int64_t b = ranges[2 * h]; b < ranges[2 * h + 1]; b += kHeavyChunk) {
      cv.push_back(hv[h]);
      cb.push_back(b);
      ce.push_back(std::min<int64_t>(b + kHeavyChunk, ranges[2 * h + 1]));
      cslot.push_back(slot0 + (int32_t)h);
    }
  }
  return PG_OK;
}

template <typename T>
int upload(T** dst, const std::vector<T>& src, hipStream_t s) {
  PG_TRY(palloc((void**)dst, sizeof(T) * std::max<size_t>(src.size(), 1)));
  if (!src.empty()) PG_HIP(hipMemcpyAsync(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, s));
  return PG_OK;
}

}  // namespace

void free_plan(VertexPlan* p) {
  pfree(p->sorted);
  pfree(p->chunk_vertex);
  pfree(p->chunk_begin);
  pfree(p->chunk_end);
  pfree(p->chunk_slot);
  pfree(p->heavy_first);
  *p = VertexPlan();
}

int build_plan(pg_graph* g, VertexPlan* P, hipStream_t s) {
  free_plan(P);
  const int32_t n = g->n;
  PG_TRY(palloc((void**)&P->sorted, sizeof(int32_t) * (size_t)std::max<int32_t>(n, 1)));
  int64_t starts[kNumBins + 1];
  PG_TRY(partition(g, true, P->sorted, starts, s));
  P->light = P->sorted + starts[1];
  P->n_light = starts[2] - starts[1];
  PG_TRY(sort_light_list(P->light, P->n_light, -1, kLightGroup * kLightUnroll, g, g->off, g->off, nullptr, s));
  {  // vertices without arcs: light, and last in the descending order
    unsigned long long* d_empty = nullptr;
    PG_TRY(dmalloc((void**)&d_empty, sizeof(unsigned long long), s));
    PG_TRY(fill_u64((uint64_t*)d_empty, 0, 1, s));
    if (n > 0) {
      hipLaunchKernelGGL(k_count_empty, dim3(grid_for(n, kBlock, INT32_MAX)), dim3(kBlock), 0, s, g->off, n, d_empty);
      PG_LAUNCH_CHECK();
    }
    unsigned long long h_empty = 0;
    PG_HIP(hipMemcpyAsync(&h_empty, d_empty, sizeof(h_empty), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    PG_TRY(dfree(d_empty, s));
    P->n_empty = (int64_t)h_empty;
  }
  P->medium = P->sorted + starts[2];
  P->n_medium = starts[3] - starts[2];
  P->n_heavy = starts[4] - starts[3];
  std::vector<int32_t> cv, cslot, first;
  std::vector<int64_t> cb, ce;
  PG_TRY(heavy_chunks(P->sorted + starts[3], P->n_heavy, g, g->off, nullptr, -1, 0, cv, cb, ce, cslot, first, s));
  first.push_back((int32_t)cv.size());
  P->n_chunks = (int64_t)cv.size();
  PG_TRY(upload(&P->chunk_vertex, cv, s));
  PG_TRY(upload(&P->chunk_begin, cb, s));
  PG_TRY(upload(&P->chunk_end, ce, s));
  PG_TRY(upload(&P->chunk_slot, cslot, s));
  PG_TRY(upload(&P->heavy_first, first, s));
  PG_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
  return PG_OK;
}

// Degrees from the offsets, the largest degree, sum_v C(d_v, 2), and the
// stable partition of the vertices by degree bin. d_maxdeg and d_wedges are
// zeroed device scratch.
static int degrees_and_bins(pg_graph* g, int* d_maxdeg, unsigned long long* d_wedges, hipStream_t s) {
  const int32_t n = g->n;
  PG_TRY(palloc((void**)&g->deg, sizeof(int32_t) * (size_t)std::max<int32_t>(n, 1)));
  if (n > 0) {
    hipLaunchKernelGGL(k_degrees, dim3(grid_for(n, kBlock, INT32_MAX)), dim3(kBlock), 0, s, g->off, n, g->deg, d_maxdeg,
                       d_wedges);
    PG_LAUNCH_CHECK();
  }
  PG_TRY(palloc((void**)&g->bin_verts, sizeof(int32_t) * (size_t)std::max<int32_t>(n, 1)));
  int64_t hbase[kNumBins + 1] = {};
  PG_TRY(partition(g, false, g->bin_verts, hbase, s));
  int h_max = 0;
  unsigned long long h_wedges = 0;
  PG_HIP(hipMemcpyAsync(&h_max, d_maxdeg, sizeof(int), hipMemcpyDeviceToHost, s));
  PG_HIP(hipMemcpyAsync(&h_wedges, d_wedges, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  PG_HIP(hipStreamSynchronize(s));
  for (int j = 0; j <= kNumBins; ++j) g->bin_start[j] = hbase[j];
  g->max_degree = h_max;
  g->wedges = h_wedges;
  return PG_OK;
}

int graph_prepare(pg_graph* g, bool validate, hipStream_t s) {
  const int32_t n = g->n;
  int* d_flags = nullptr;
  int* d_maxdeg = nullptr;
  unsigned long long* d_wedges = nullptr;
  PG_TRY(dmalloc((void**)&d_flags, 64, s));
  d_maxdeg = d_flags + 1;
  d_wedges = (unsigned long long*)(d_flags + 2);
  PG_HIP(hipMemsetAsync(d_flags, 0, 64, s));

  // 1. bounds: offsets monotone in [0, nnz], IDs in [0, n). After this every
  //    later kernel's indexing stays inside the arrays.
  hipLaunchKernelGGL(k_check_offsets, dim3(grid_for((int64_t)n + 1, kBlock, INT32_MAX)), dim3(kBlock), 0, s, g->off, n, g->nnz,
                     d_flags);
  PG_LAUNCH_CHECK();
  int h_flags = 0;
  PG_HIP(hipMemcpyAsync(&h_flags, d_flags, sizeof(int), hipMemcpyDeviceToHost, s));
  PG_HIP(hipStreamSynchronize(s));
  if (h_flags) {
    dfree(d_flags, s);
    return fail(PG_E_GRAPH, "CSR offsets are not a monotone sequence from 0 to nnz");
  }
  if (g->nnz > 0) {
    hipLaunchKernelGGL(k_check_range, dim3(grid_for(g->nnz, kBlock, 8192)), dim3(kBlock), 0, s, g->adj, g->nnz, n,
                       d_flags);
    PG_LAUNCH_CHECK();
  }
  if (validate && g->nnz > 0) {
    PG_HIP(hipMemcpyAsync(&h_flags, d_flags, sizeof(int), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    if (h_flags == 0) {
      hipLaunchKernelGGL(k_check_structure, dim3(grid_for(g->nnz, kBlock, 8192)), dim3(kBlock), 0, s, g->off, g->adj,
                         n, g->nnz, d_flags);
      PG_LAUNCH_CHECK();
    }
  }
  PG_HIP(hipMemcpyAsync(&h_flags, d_flags, sizeof(int), hipMemcpyDeviceToHost, s));
  PG_HIP(hipStreamSynchronize(s));
  if (h_flags) {
    dfree(d_flags, s);
    std::string why;
    if (h_flags & kBadRange) why += " neighbour ID out of range;";
    if (h_flags & kSelfLoop) why += " self-loop;";
    if (h_flags & kUnsorted) why += " neighbourhood not strictly ascending (unsorted or duplicate);";
    if (h_flags & kAsymmetric) why += " not symmetric;";
    return fail(PG_E_GRAPH, "CSR rejected:" + why);
  }

  // 2-3. degrees, max degree, wedge count, degree bins
  PG_TRY(degrees_and_bins(g, d_maxdeg, d_wedges, s));

  // 4. upper edges: ustart, upper-edge offsets, (eu, ev) in CSR order
  int64_t* up = nullptr;
  PG_TRY(dmalloc((void**)&up, sizeof(int64_t) * ((size_t)n + 1), s));
  PG_TRY(palloc((void**)&g->ustart, sizeof(int32_t) * (size_t)std::max<int32_t>(n, 1)));
  PG_TRY(palloc((void**)&g->upoff, sizeof(int64_t) * ((size_t)n + 1)));
  PG_HIP(hipMemsetAsync(up, 0, sizeof(int64_t) * ((size_t)n + 1), s));
  PG_FOR_BINS(k_upper_count, g, s, g->off, g->adj, verts_, cnt_, up, g->ustart);
  PG_TRY(exclusive_scan_i64(up, g->upoff, (int64_t)n + 1, s));
  int64_t m = 0;
  PG_HIP(hipMemcpyAsync(&m, g->upoff + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  PG_HIP(hipStreamSynchronize(s));
  g->m = m;
  PG_TRY(palloc((void**)&g->eu, sizeof(int32_t) * (size_t)std::max<int64_t>(m, 1)));
  PG_TRY(palloc((void**)&g->ev, sizeof(int32_t) * (size_t)std::max<int64_t>(m, 1)));
  PG_FOR_BINS(k_upper_fill, g, s, g->off, g->adj, verts_, cnt_, g->upoff, g->eu, g->ev);
  PG_TRY(dfree(up, s));
  PG_TRY(dfree(d_flags, s));

  // 5. work plans over N_v and over the upper neighbours
  PG_TRY(build_plan(g, &g->plan_all, s));
  return PG_OK;
}

int graph_arc_sources(pg_graph* g, hipStream_t s) {
  if (g->arc_src) return PG_OK;
  PG_TRY(palloc((void**)&g->arc_src, sizeof(int32_t) * (size_t)std::max<int64_t>(g->nnz, 1)));
  PG_FOR_BINS(k_arc_src, g, s, g->off, verts_, cnt_, g->arc_src);
  return PG_OK;
}

int graph_orient(pg_graph* g, hipStream_t s) {
  if (g->poff) return PG_OK;
  ProfScope ps(s, "orient");
  const int32_t n = g->n;
  int64_t* cnt = nullptr;
  PG_TRY(dmalloc((void**)&cnt, sizeof(int64_t) * 2 * ((size_t)n + 1), s));
  int64_t* poff64 = cnt + (n + 1);
  PG_HIP(hipMemsetAsync(cnt, 0, sizeof(int64_t) * ((size_t)n + 1), s));
  PG_FOR_BINS(k_orient_count, g, s, g->off, g->adj, g->deg, verts_, cnt_, cnt);
  PG_TRY(exclusive_scan_i64(cnt, poff64, (int64_t)n + 1, s));
  PG_TRY(palloc((void**)&g->padj, sizeof(int32_t) * (size_t)std::max<int64_t>(g->m, 1)));
  PG_TRY(palloc((void**)&g->parc_src, sizeof(int32_t) * (size_t)std::max<int64_t>(g->m, 1)));
  for (int bin = 0; bin < kNumBins; ++bin) {
    const int64_t cnt_v = g->bin_start[bin + 1] - g->bin_start[bin];
    if (cnt_v <= 0) continue;
    const int32_t* verts = g->bin_verts + g->bin_start[bin];
    const int G = std::min(kBinGroup[bin], kWave);
    const unsigned grid = (unsigned)((cnt_v * G + kBlock - 1) / kBlock);
    if (G == 4)
      hipLaunchKernelGGL(k_orient_fill<4>, dim3(grid), dim3(kBlock), 0, s, g->off, g->adj, g->deg, verts, cnt_v,
                         poff64, g->padj, g->parc_src);
    else if (G == 16)
      hipLaunchKernelGGL(k_orient_fill<16>, dim3(grid), dim3(kBlock), 0, s, g->off, g->adj, g->deg, verts, cnt_v,
                         poff64, g->padj, g->parc_src);
    else
      hipLaunchKernelGGL(k_orient_fill<64>, dim3(grid), dim3(kBlock), 0, s, g->off, g->adj, g->deg, verts, cnt_v,
                         poff64, g->padj, g->parc_src);
    PG_LAUNCH_CHECK();
  }
  PG_TRY(palloc((void**)&g->poff, sizeof(int32_t) * ((size_t)n + 1)));
  hipLaunchKernelGGL(k_i64_to_i32, dim3(grid_for((int64_t)n + 1, kBlock, 4096)), dim3(kBlock), 0, s, poff64, g->poff,
                     (int64_t)n + 1);
  PG_LAUNCH_CHECK();
  return dfree(cnt, s);
}

int graph_oriented(pg_graph* g, hipStream_t s) {
  if (g->oriented) return PG_OK;
  PG_TRY(graph_orient(g, s));
  pg_graph* o = new (std::nothrow) pg_graph();
  if (!o) return fail(PG_E_NOMEM, "host allocation failed");
  o->ctx = g->ctx;
  o->n = g->n;
  o->nnz = g->m;  // every undirected edge once, at its lower-ranked end
  o->owns_csr = false;
  o->off = g->poff;
  o->adj = g->padj;
  int* d_scratch = nullptr;
  int rc = dmalloc((void**)&d_scratch, 64, s);
  if (rc == PG_OK && hipMemsetAsync(d_scratch, 0, 64, s) != hipSuccess) rc = fail(PG_E_DEVICE, "hipMemsetAsync failed");
  if (rc == PG_OK) rc = degrees_and_bins(o, d_scratch + 1, (unsigned long long*)(d_scratch + 2), s);
  if (rc == PG_OK) rc = build_plan(o, &o->plan_all, s);
  if (d_scratch) dfree(d_scratch, s);
  if (rc != PG_OK) {
    (void)hipStreamSynchronize(s);
    pfree(o->deg);
    pfree(o->bin_verts);
    free_plan(&o->plan_all);
    delete o;
    return rc;
  }
  g->oriented = o;
  return PG_OK;
}

void free_slabs(SlabPlan* p) {
  pfree(p->split);
  pfree(p->verts);
  pfree(p->chunk_vertex);
  pfree(p->chunk_begin);
  pfree(p->chunk_end);
  pfree(p->rank);
  pfree(p->chunk_ptr);
  pfree(p->chunk_list);
  *p = SlabPlan();
}

namespace {

// A slab plan over the arcs [begin[v], off[v+1]) of every vertex: the upper
// neighbours (begin = ustart, the triangle count) or all of N_v (begin = off,
// the clustering coefficient, which also gets the sliced vertices' ranks and
// chunk lists).
int build_slabs(pg_graph* g, const int32_t* begin, bool all, SlabPlan* out, hipStream_t s) {
  const int32_t n = g->n;
  SlabPlan Q;  // filled here, moved into the graph once complete
  int rc = [&]() -> int {
    // 1. boundaries by incoming sliced arcs, 2. per-vertex split positions
    int64_t* cnt = nullptr;
    PG_TRY(dmalloc((void**)&cnt, sizeof(int64_t) * 2 * (size_t)n + 16 * sizeof(int32_t), s));
    int64_t* pre = cnt + n;
    int32_t* lo = (int32_t*)(pre + n);
    PG_TRY(fill_u64((uint64_t*)cnt, 0, n, s));
    PG_FOR_BINS(k_in_sliced, g, s, g->off, begin, g->adj, verts_, cnt_, (unsigned long long*)cnt);
    PG_TRY(exclusive_scan_i64(cnt, pre, n, s));
    hipLaunchKernelGGL(k_slab_bounds, dim3(1), dim3(64), 0, s, (const int64_t*)pre, (const int64_t*)cnt, n, lo);
    PG_LAUNCH_CHECK();
    PG_TRY(palloc((void**)&Q.split, sizeof(int32_t) * (size_t)(kSlabs - 1) * (size_t)n));
    hipLaunchKernelGGL(k_slab_split, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, s, g->off, begin, g->adj, n,
                       (const int32_t*)lo, Q.split);
    PG_LAUNCH_CHECK();
    PG_TRY(dfree(cnt, s));
    // 3. item tiers slab by slab, then the whole vertices
    const int64_t nk = (int64_t)(kSlabs + 1) * n;
    uint8_t* keys = nullptr;
    int32_t* sorted = nullptr;
    PG_TRY(dmalloc((void**)&keys, (size_t)nk, s));
    PG_TRY(dmalloc((void**)&sorted, sizeof(int32_t) * (size_t)nk, s));
    hipLaunchKernelGGL(k_slab_keys, dim3((unsigned)((nk + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, g->off, begin,
                       (const int32_t*)Q.split, n, keys);
    PG_LAUNCH_CHECK();
    int64_t st[kSlabs + 1][kNumBins + 1];
    int64_t lists = 0;
    for (int x = 0; x <= kSlabs; ++x) {
      PG_TRY(partition_keys(keys + (size_t)x * n, n, sorted + (size_t)x * n, st[x], s));
      lists += st[x][3] - st[x][1];
    }
    // 4. light and medium lists of every slab, then the whole vertices
    PG_TRY(palloc((void**)&Q.verts, sizeof(int32_t) * (size_t)std::max<int64_t>(lists, 1)));
    int64_t at = 0;
    for (int x = 0; x <= kSlabs; ++x) {
      const int64_t cnt_x = st[x][3] - st[x][1];
      if (x < kSlabs) {
        Q.light_at[x] = at;
        Q.n_light[x] = st[x][2] - st[x][1];
        Q.medium_at[x] = at + Q.n_light[x];
        Q.n_medium[x] = st[x][3] - st[x][2];
      } else {
        Q.whole_at = at;
        Q.n_whole = cnt_x;
      }
      if (cnt_x > 0)
        PG_HIP(hipMemcpyAsync(Q.verts + at, sorted + (size_t)x * n + st[x][1], sizeof(int32_t) * cnt_x,
                              hipMemcpyDeviceToDevice, s));
      at += cnt_x;
    }
    for (int x = 0; x < kSlabs; ++x)
      PG_TRY(sort_light_list(Q.verts + Q.light_at[x], Q.n_light[x], x, kSlabLightBucket, g, g->off, begin, Q.split,
                             s));
    PG_TRY(sort_light_list(Q.verts + Q.whole_at, Q.n_whole, -1, kSlabWholeBucket, g, g->off, begin, Q.split, s));
    // 5. heavy items in chunks
    std::vector<int32_t> cv, cslot, first;
    std::vector<int64_t> cb, ce;
    for (int x = 0; x < kSlabs; ++x) {
      Q.chunk_at[x] = (int64_t)cv.size();
      PG_TRY(heavy_chunks(sorted + (size_t)x * n + st[x][3], st[x][4] - st[x][3], g, begin, Q.split, x, 0, cv, cb, ce,
                          cslot, first, s));
      Q.n_chunks[x] = (int64_t)cv.size() - Q.chunk_at[x];
    }
    int64_t busiest = 0;
    for (int x = 0; x < kSlabs; ++x) busiest = std::max(busiest, slab_blocks(Q, x));
    Q.slab_grid = busiest * kSlabs;
    PG_TRY(upload(&Q.chunk_vertex, cv, s));
    PG_TRY(upload(&Q.chunk_begin, cb, s));
    PG_TRY(upload(&Q.chunk_end, ce, s));
    std::vector<int32_t> cptr, clist;
    if (all) {
      // 6. ranks of the sliced vertices, and each one's chunks (whatever slab they are in)
      int64_t* flag = nullptr;
      PG_TRY(dmalloc((void**)&flag, sizeof(int64_t) * 2 * (size_t)n, s));
      int64_t* pre = flag + n;
      hipLaunchKernelGGL(k_sliced_flags, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, g->off, begin,
                         n, flag);
      PG_LAUNCH_CHECK();
      PG_TRY(exclusive_scan_i64(flag, pre, n, s));
      PG_TRY(palloc((void**)&Q.rank, sizeof(int32_t) * (size_t)n));
      hipLaunchKernelGGL(k_sliced_rank, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                         (const int64_t*)flag, (const int64_t*)pre, n, Q.rank);
      PG_LAUNCH_CHECK();
      std::vector<int32_t> rank_h((size_t)n);
      int64_t last[2] = {0, 0};
      PG_HIP(hipMemcpyAsync(rank_h.data(), Q.rank, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s));
      PG_HIP(hipMemcpyAsync(&last[0], flag + (n - 1), sizeof(int64_t), hipMemcpyDeviceToHost, s));
      PG_HIP(hipMemcpyAsync(&last[1], pre + (n - 1), sizeof(int64_t), hipMemcpyDeviceToHost, s));
      PG_HIP(hipStreamSynchronize(s));
      PG_TRY(dfree(flag, s));
      Q.n_sliced = last[0] + last[1];
      cptr.assign((size_t)Q.n_sliced + 1, 0);
      for (int32_t v : cv) {
        const int32_t r = rank_h[(size_t)v];
        if (r < 0) return fail(PG_E_DEVICE, "slab plan: a chunk of a vertex that is not sliced");
        ++cptr[(size_t)r + 1];
      }
      for (int64_t r = 0; r < Q.n_sliced; ++r) cptr[(size_t)r + 1] += cptr[(size_t)r];
      clist.assign(cv.size(), 0);
      std::vector<int32_t> fill(cptr.begin(), cptr.end() - 1);
      for (size_t c = 0; c < cv.size(); ++c) clist[(size_t)fill[(size_t)rank_h[(size_t)cv[c]]]++] = (int32_t)c;
      PG_TRY(upload(&Q.chunk_ptr, cptr, s));
      PG_TRY(upload(&Q.chunk_list, clist, s));
    }
    PG_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
    PG_TRY(dfree(sorted, s));
    return dfree(keys, s);
  }();
  if (rc != PG_OK) {
    free_slabs(&Q);
    return rc;
  }
  *out = Q;
  return PG_OK;
}

}  // namespace

int graph_slabs(pg_graph* g, hipStream_t s) {
  if (g->slabs.split || g->n == 0) return PG_OK;
  ProfScope ps(s, "slabs");
  return build_slabs(g, g->ustart, false, &g->slabs, s);
}

int graph_slabs_all(pg_graph* g, hipStream_t s) {
  if (g->slabs_all.split || g->n == 0) return PG_OK;
  ProfScope ps(s, "slabs");
  return build_slabs(g, g->off, true, &g->slabs_all, s);
}

}  // namespace pg
