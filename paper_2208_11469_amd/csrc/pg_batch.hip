// Batched small graphs: per-graph Bloom filters, clustering coefficients and
// triangle counts for many graphs in persistent launches.
//
// Layout (one arena for all graphs): global vertex IDs vbase[g] + v, int64
// arc offsets over all graphs, neighbour IDs kept local to their graph, filter
// rows of graph g at word wbase[g] + v * W[g], estimator tables at tbase[g].
//
// Work list (built on the host, heaviest first): a heavy vertex (more than
// kBatchHeavy arcs) is one item processed by a whole block; the other vertices
// form tiles of tile_vertices consecutive vertices, kBatchGroup lanes per
// vertex. Persistent blocks take items from a counter reset at the start of
// every run and leave when the list is exhausted. The estimate runs one
// launch per row width W present (its items grouped by W), so W is a
// compile-time constant of that launch; the launches are dealt to four
// streams (longest first, each to the least-loaded stream) so that their
// tails overlap, and a captured run keeps them as parallel graph branches.
// Within a width, each graph belongs to one XCD (dealt longest first to the
// least-loaded one): block i runs on XCD i mod 8 and takes items only from
// that XCD's queue, so a graph's rows are gathered through one L2.
//
// No block ever waits for another block: a block leaves as soon as the index
// it draws from its queue counter is past the end of its list, every loop is
// bounded by the list or the vertex's arcs, and every barrier sits where the
// whole block takes the same branch (the drawn index and the item are read
// from LDS after a barrier). So every launch ends whatever the number of
// resident blocks.
//
// Each vertex is always reduced by the same lanes in the same order (its tier
// is fixed by its degree), so results do not depend on the tile size, the grid
// size or which block took which item.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "pg_device.h"
#include "pg_internal.h"

namespace pg {
namespace {

constexpr int kBlock = 256;
constexpr int kBatchGroup = 8;
constexpr int kGroups = kBlock / kBatchGroup;
constexpr int32_t kBatchHeavy = 512;
constexpr int kMaxW = 16;

struct GraphDesc {
  int64_t vbase;  // first global vertex
  int64_t wbase;  // first word of the graph's rows
  int64_t tbase;  // first entry of the graph's estimator table
  int32_t n;
  uint32_t B;
  uint32_t W;
  int32_t pad;
};

// The estimate items of one row width, split by XCD: XCD x takes
// eitems[at[x] .. at[x + 1]).
struct XQueues {
  int64_t at[kSlabs + 1];
};

struct Item {
  int32_t graph;
  int32_t heavy;  // 1: the single vertex v0 with a whole block
  int32_t v0, v1; // local vertex range
};

struct BatchView {
  const GraphDesc* gd;
  const Item* items;
  int64_t nitems;
  const int64_t* off;
  const int32_t* adj;
  uint64_t* words;
  uint32_t* pc;
  const uint64_t* ha;
  const uint64_t* hc;
  uint32_t b;
  const double* tables;
  double* S;
  double* Splus;
  float* cc;
  uint32_t* counters;  // [0] build queue, [1 + W * kSlabs + x] estimate queue of row width W on XCD x
};

// [0] the build queue, then per row width W one estimate queue per XCD
// (slab): counter 1 + W * kSlabs + x
constexpr int kCounters = 1 + (kMaxW + 1) * kSlabs;
constexpr int kBranches = 4;  // concurrent estimate streams (the box's hardware queues per process)

__global__ void k_batch_reset(uint32_t* counters) {
  for (int i = threadIdx.x; i < kCounters; i += blockDim.x) counters[i] = 0;
}

// One block per graph: T_g[c] for c = 0..B_g (same formulas as the single-graph tables).
__global__ void k_batch_tables(const GraphDesc* __restrict__ gd, uint32_t b, int est, double* __restrict__ tables) {
  const GraphDesc d = gd[blockIdx.x];
  const double Bd = (double)d.B, bd = (double)b;
  for (uint32_t c = threadIdx.x; c <= d.B; c += blockDim.x) {
    const double ct = (double)(c == d.B ? c - 1 : c);
    double r;
    if (est == PG_EST_BF_AND)
      r = -(Bd / bd) * log(1.0 - ct / Bd);
    else if (est == PG_EST_BF_L)
      r = (double)c / bd;
    else
      r = log(1.0 - ct / Bd) / (bd * log(1.0 - 1.0 / Bd));
    tables[d.tbase + c] = r;
  }
}

__device__ __forceinline__ int64_t next_item(uint32_t* counter, int64_t* slot) {
  if (threadIdx.x == 0) *slot = (int64_t)atomicAdd(counter, 1u);
  __syncthreads();
  const int64_t it = *slot;
  __syncthreads();
  return it;
}

// Bits of the neighbours adj[beg, end) into `bits`, G lanes: LDS atomic OR,
// which is order-independent, so the row does not depend on which lane
// lands first.
__device__ __forceinline__ void scatter_arcs(const BatchView& bv, int64_t beg, int64_t end, int lane, int G,
                                             uint32_t B, uint64_t* __restrict__ bits) {
  for (int64_t p0 = beg + lane; p0 < end; p0 += (int64_t)G * 4) {
    uint32_t x[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t p = p0 + (int64_t)j * G;
      x[j] = p < end ? (uint32_t)bv.adj[p] : 0u;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (p0 + (int64_t)j * G < end) {
        for (uint32_t i = 0; i < bv.b; ++i) {
          const uint32_t idx = bf_index(bv.ha[i], bv.hc[i], x[j], B);
          atomicOr((unsigned long long*)&bits[idx >> 6], 1ull << (idx & 63u));
        }
      }
    }
  }
}

// LDS visibility among the lanes of one wave.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Heavy items: the block shares kBuildCopies bitmaps (lane l uses copy
// l mod kBuildCopies, so fewer lanes of one instruction collide on a word);
// tiles: each group of kBatchGroup lanes shares one bitmap per vertex.
constexpr int kBuildCopies = 8;
constexpr int kBuildWords = (kGroups > kBuildCopies ? kGroups : kBuildCopies) * kMaxW;

__global__ __launch_bounds__(kBlock) void k_batch_build(BatchView bv) {
  __shared__ uint64_t lds[kBuildWords];
  __shared__ uint32_t ones_sh[kMaxW];
  __shared__ int64_t slot;
  const int tid = threadIdx.x;
  for (;;) {
    const int64_t it = next_item(&bv.counters[0], &slot);
    if (it >= bv.nitems) return;
    const Item item = bv.items[it];
    const GraphDesc gd = bv.gd[item.graph];
    const uint32_t W = gd.W;
    if (item.heavy) {
      for (uint32_t i = tid; i < kBuildCopies * W; i += kBlock) lds[i] = 0;
      __syncthreads();
      const int64_t gv = gd.vbase + item.v0;
      scatter_arcs(bv, bv.off[gv], bv.off[gv + 1], tid, kBlock, gd.B, lds + (tid % kBuildCopies) * W);
      __syncthreads();
      if ((uint32_t)tid < W) {
        uint64_t w = 0;
#pragma unroll
        for (int c = 0; c < kBuildCopies; ++c) w |= lds[c * W + tid];
        bv.words[gd.wbase + (int64_t)item.v0 * W + tid] = w;
        ones_sh[tid] = (uint32_t)__popcll(w);
      }
      __syncthreads();
      if (tid == 0) {
        uint32_t ones = 0;
        for (uint32_t k = 0; k < W; ++k) ones += ones_sh[k];
        bv.pc[gv] = ones;
      }
      __syncthreads();
      continue;
    }
    const int grp = tid / kBatchGroup, lane = tid % kBatchGroup;
    uint64_t* bits = lds + grp * kMaxW;
    for (int32_t v = item.v0 + grp; v < item.v1; v += kGroups) {
      const int64_t gv = gd.vbase + v;
      const int64_t beg = bv.off[gv], end = bv.off[gv + 1];
      if (end - beg > kBatchHeavy) continue;  // a heavy item of its own
      for (uint32_t k = lane; k < W; k += kBatchGroup) bits[k] = 0;
      wave_sync();
      scatter_arcs(bv, beg, end, lane, kBatchGroup, gd.B, bits);
      wave_sync();
      uint32_t ones = 0;
      for (uint32_t k = lane; k < W; k += kBatchGroup) {
        const uint64_t w = bits[k];
        bv.words[gd.wbase + (int64_t)v * W + k] = w;
        ones += (uint32_t)__popcll(w);
      }
      ones = group_sum_u32<kBatchGroup>(ones);
      if (lane == 0) bv.pc[gv] = ones;
      wave_sync();  // before the next vertex clears the bitmap
    }
    __syncthreads();
  }
}

// Sums of the estimate over the arcs of v (all, and those to larger IDs) for a
// group of G lanes, rows of W words. v's row stays in registers; a neighbour's
// row is read by a team of T lanes side by side (Q words each; the last member
// may read up to Q - 1 words past the row, which the zero words of v's row
// cancel), and the team's counts meet in quad DPP adds.
template <int W, int G>
__device__ __forceinline__ void vertex_sums(const BatchView& bv, const GraphDesc& gd, int32_t v, int64_t beg,
                                            int64_t end, int lane, double& all, double& up) {
  constexpr int T = W <= 2 ? 1 : 2;
  constexpr int Q = (W + T - 1) / T;
  constexpr int NT = G / T;
  constexpr int U = W <= 4 ? 8 : (W <= 8 ? 4 : 2);
  const int k = lane % T;
  const bool reads = k * Q < W;
  const uint64_t* rows = bv.words + gd.wbase;
  uint64_t rv[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) rv[i] = (k * Q + i < W) ? rows[(int64_t)v * W + k * Q + i] : 0ull;
  const double* tab = bv.tables + gd.tbase;
  for (int64_t p0 = beg + lane / T; p0 < end; p0 += (int64_t)NT * U) {
    int32_t x[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int64_t p = p0 + (int64_t)j * NT;
      x[j] = p < end ? bv.adj[p] : -1;
    }
    uint64_t w[U][Q];
#pragma unroll
    for (int j = 0; j < U; ++j) {
#pragma unroll
      for (int i = 0; i < Q; ++i) w[j][i] = 0;
      if (x[j] >= 0 && reads) {
        const uint64_t* r = rows + (int64_t)x[j] * W + k * Q;
#pragma unroll
        for (int i = 0; i < Q; ++i) w[j][i] = r[i];
      }
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      uint32_t c = 0;
#pragma unroll
      for (int i = 0; i < Q; ++i) c += (uint32_t)__popcll(rv[i] & w[j][i]);
      c = team_sum<T>(c);
      if (k == 0 && x[j] >= 0) {
        const double t = tab[c];
        all += t;
        if (x[j] > v) up += t;
      }
    }
  }
}

// Estimate items [begin, end) of one row width W (graphs with B = 64 W).
template <int W>
__global__ __launch_bounds__(kBlock) void k_batch_estimate(BatchView bv, XQueues q) {
  __shared__ double red[kBlock / kWave];
  __shared__ int64_t slot;
  const int tid = threadIdx.x;
  const int x = (int)(blockIdx.x % kSlabs);  // the XCD the block runs on: it takes that XCD's graphs
  for (;;) {
    const int64_t it = q.at[x] + next_item(&bv.counters[1 + W * kSlabs + x], &slot);
    if (it >= q.at[x + 1]) return;
    const Item item = bv.items[it];
    const GraphDesc gd = bv.gd[item.graph];
    if (item.heavy) {
      const int64_t gv = gd.vbase + item.v0;
      double all = 0.0, up = 0.0;
      vertex_sums<W, kBlock>(bv, gd, item.v0, bv.off[gv], bv.off[gv + 1], tid, all, up);
      all = block_sum_256(all, red);
      up = block_sum_256(up, red);
      if (tid == 0) {
        const int64_t d = bv.off[gv + 1] - bv.off[gv];
        bv.S[gv] = all;
        bv.Splus[gv] = up;
        bv.cc[gv] = d >= 2 ? (float)(all / ((double)d * ((double)d - 1.0))) : 0.0f;
      }
      continue;
    }
    const int grp = tid / kBatchGroup, lane = tid % kBatchGroup;
    for (int32_t v = item.v0 + grp; v < item.v1; v += kGroups) {
      const int64_t gv = gd.vbase + v;
      const int64_t beg = bv.off[gv], e = bv.off[gv + 1];
      if (e - beg > kBatchHeavy) continue;
      double all = 0.0, up = 0.0;
      vertex_sums<W, kBatchGroup>(bv, gd, v, beg, e, lane, all, up);
      all = group_sum<kBatchGroup>(all);
      up = group_sum<kBatchGroup>(up);
      if (lane == 0) {
        const int64_t d = e - beg;
        bv.S[gv] = all;
        bv.Splus[gv] = up;
        bv.cc[gv] = d >= 2 ? (float)(all / ((double)d * ((double)d - 1.0))) : 0.0f;
      }
    }
  }
}

// One block per graph: TC_g = (1/3) sum of the upper sums, fixed order.
// Thread t adds entries t, t + 256, ... in rounds of kTcLoads independent
// loads into kTcLoads accumulators (the largest graphs have 2^16 vertices:
// one load in flight per thread took 0.1 ms), then a fixed tree.
constexpr int kTcLoads = 8;
__global__ __launch_bounds__(kBlock) void k_batch_tc(const GraphDesc* __restrict__ gd,
                                                     const double* __restrict__ Splus, double* __restrict__ tc) {
  __shared__ double red[kBlock / kWave];
  const GraphDesc d = gd[blockIdx.x];
  double a[kTcLoads];
#pragma unroll
  for (int j = 0; j < kTcLoads; ++j) a[j] = 0.0;
  for (int32_t v0 = threadIdx.x; v0 < d.n; v0 += kBlock * kTcLoads) {
    double x[kTcLoads];
#pragma unroll
    for (int j = 0; j < kTcLoads; ++j) {
      const int32_t v = v0 + j * kBlock;
      x[j] = v < d.n ? Splus[d.vbase + v] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kTcLoads; ++j) a[j] += x[j];
  }
  const double acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  const double r = block_sum_256(acc, red);
  if (threadIdx.x == 0) tc[blockIdx.x] = r / 3.0;
}

}  // namespace
}  // namespace pg

struct pg_batch {
  pg_ctx* ctx = nullptr;
  int32_t count = 0;
  int64_t N = 0;       // vertices over all graphs
  int64_t arcs = 0;
  uint32_t b = 1;
  uint64_t seed = 0;
  pg_batch_params params{64, 4};
  std::vector<pg::GraphDesc> h_gd;
  std::vector<int64_t> h_off;  // host copy of the global offsets (work-list construction)
  pg::GraphDesc* gd = nullptr;
  pg::Item* items = nullptr;   // build work list (heaviest first)
  int64_t items_cap = 0;
  int64_t nitems = 0;
  pg::Item* eitems = nullptr;  // estimate work list: by row width W, heaviest first inside
  int64_t w_begin[pg::kMaxW + 2] = {};  // items of width W: eitems[w_begin[W] .. w_begin[W + 1])
  pg::XQueues xq[pg::kMaxW + 1] = {};   // of those, XCD x's: eitems[xq[W].at[x] .. xq[W].at[x + 1])
  int64_t* off = nullptr;
  int32_t* adj = nullptr;
  uint64_t* words = nullptr;
  uint32_t* pc = nullptr;
  uint64_t* ha = nullptr;
  uint64_t* hc = nullptr;
  double* tables = nullptr;
  double* S = nullptr;
  double* Splus = nullptr;
  float* cc = nullptr;
  double* tc = nullptr;
  uint32_t* counters = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // the per-width estimate launches are dealt to kBranches streams: the
  // caller's and these (default priority), forked after the build and joined
  // before the triangle-count sums
  hipStream_t side[pg::kBranches - 1] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[pg::kBranches - 1] = {};
  int branch_of[pg::kMaxW + 1] = {};  // stream of each row width's launch (0 = the caller's)
  int launch_order[pg::kMaxW] = {};   // row widths by descending work
  int n_widths = 0;
};

namespace pg {
namespace {

int build_items(pg_batch* bt) {
  const int32_t T = bt->params.tile_vertices;
  std::vector<std::pair<int64_t, Item>> list;
  for (int32_t g = 0; g < bt->count; ++g) {
    const GraphDesc& d = bt->h_gd[g];
    for (int32_t v0 = 0; v0 < d.n; v0 += T) {
      const int32_t v1 = std::min(d.n, v0 + T);
      int64_t cost = 0;
      for (int32_t v = v0; v < v1; ++v) {
        const int64_t deg = bt->h_off[d.vbase + v + 1] - bt->h_off[d.vbase + v];
        if (deg > kBatchHeavy)
          list.push_back({deg, Item{g, 1, v, v + 1}});
        else
          cost += deg + 1;
      }
      list.push_back({cost, Item{g, 0, v0, v1}});
    }
  }
  std::stable_sort(list.begin(), list.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
  std::vector<Item> items(list.size()), eitems;
  for (size_t i = 0; i < list.size(); ++i) items[i] = list[i].second;
  eitems.reserve(items.size());
  // graphs of each row width dealt to the XCDs longest first, each to the
  // XCD with the least work so far, so that a graph's rows stay in one L2
  std::vector<int64_t> gcost((size_t)bt->count, 0);
  for (const auto& pr : list) gcost[(size_t)pr.second.graph] += pr.first;
  std::vector<int32_t> gorder((size_t)bt->count);
  for (int32_t g = 0; g < bt->count; ++g) gorder[(size_t)g] = g;
  std::stable_sort(gorder.begin(), gorder.end(), [&](int32_t a, int32_t b) { return gcost[(size_t)a] > gcost[(size_t)b]; });
  std::vector<int8_t> gxcd((size_t)bt->count, 0);
  int64_t xload[kMaxW + 1][kSlabs] = {};
  for (int32_t g : gorder) {
    int64_t* ld = xload[bt->h_gd[g].W];
    const int x = (int)(std::min_element(ld, ld + kSlabs) - ld);
    ld[x] += gcost[(size_t)g];
    gxcd[(size_t)g] = (int8_t)x;
  }
  for (int w = 0; w <= kMaxW + 1; ++w) bt->w_begin[w] = 0;
  for (uint32_t w = 1; w <= (uint32_t)kMaxW; ++w) {  // stable: heaviest first inside a queue
    bt->w_begin[w] = (int64_t)eitems.size();
    for (int x = 0; x < kSlabs; ++x) {
      bt->xq[w].at[x] = (int64_t)eitems.size();
      for (const Item& it : items)
        if (bt->h_gd[it.graph].W == w && gxcd[(size_t)it.graph] == x) eitems.push_back(it);
    }
    bt->xq[w].at[kSlabs] = (int64_t)eitems.size();
  }
  bt->w_begin[kMaxW + 1] = (int64_t)eitems.size();
  // work per row width (arcs times the row words each arc reads, plus one
  // per vertex), dealt to the branches longest first, each to the branch with
  // the least work so far
  int64_t cost[kMaxW + 1] = {};
  for (const auto& pr : list) cost[bt->h_gd[pr.second.graph].W] += pr.first * (int64_t)(bt->h_gd[pr.second.graph].W + 1);
  std::vector<int> order;
  for (int w = 1; w <= kMaxW; ++w)
    if (bt->w_begin[w + 1] > bt->w_begin[w]) order.push_back(w);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  int64_t load[kBranches] = {};
  bt->n_widths = (int)order.size();
  for (size_t i = 0; i < order.size(); ++i) {
    const int br = (int)(std::min_element(load, load + kBranches) - load);
    load[br] += cost[order[i]];
    bt->branch_of[order[i]] = br;
    bt->launch_order[i] = order[i];
  }
  if ((int64_t)items.size() > bt->items_cap) {
    pfree(bt->items);
    pfree(bt->eitems);
    bt->items = nullptr;
    bt->eitems = nullptr;
    bt->items_cap = (int64_t)items.size();
    PG_TRY(palloc((void**)&bt->items, sizeof(Item) * std::max<size_t>(items.size(), 1)));
    PG_TRY(palloc((void**)&bt->eitems, sizeof(Item) * std::max<size_t>(items.size(), 1)));
  }
  bt->nitems = (int64_t)items.size();
  if (!items.empty()) {
    PG_HIP(hipMemcpy(bt->items, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice));
    PG_HIP(hipMemcpy(bt->eitems, eitems.data(), sizeof(Item) * eitems.size(), hipMemcpyHostToDevice));
  }
  return PG_OK;
}

BatchView view_of(pg_batch* bt) {
  BatchView v;
  v.gd = bt->gd;
  v.items = bt->items;
  v.nitems = bt->nitems;
  v.off = bt->off;
  v.adj = bt->adj;
  v.words = bt->words;
  v.pc = bt->pc;
  v.ha = bt->ha;
  v.hc = bt->hc;
  v.b = bt->b;
  v.tables = bt->tables;
  v.S = bt->S;
  v.Splus = bt->Splus;
  v.cc = bt->cc;
  v.counters = bt->counters;
  return v;
}

// The whole run: kernels only, no allocation and no memset (capturable).
int enqueue_run(pg_batch* bt, int est, hipStream_t s) {
  ProfScope ps(s, "batch_run");
  const BatchView bv = view_of(bt);
  const unsigned persistent = (unsigned)std::max<int64_t>(
      1, std::min<int64_t>(bt->nitems, (int64_t)std::max(1, bt->ctx->num_cus) * bt->params.blocks_per_cu));
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(kBlock), 0, s, bt->counters);
  PG_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_batch_tables, dim3((unsigned)bt->count), dim3(kBlock), 0, s, (const GraphDesc*)bt->gd, bt->b,
                     est, bt->tables);
  PG_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_batch_build, dim3(persistent), dim3(kBlock), 0, s, bv);
  PG_LAUNCH_CHECK();
  BatchView ev = bv;
  ev.items = bt->eitems;
  // the estimate launches on kBranches streams, ordered after the build and
  // before the sums by events (these become graph edges under capture)
  PG_HIP(hipEventRecord(bt->fork, s));
  for (int i = 0; i < kBranches - 1; ++i) PG_HIP(hipStreamWaitEvent(bt->side[i], bt->fork, 0));
  for (int i = 0; i < bt->n_widths; ++i) {
    const int w = bt->launch_order[i];
    const int64_t b0 = bt->w_begin[w], b1 = bt->w_begin[w + 1];
    const hipStream_t ws = bt->branch_of[w] == 0 ? s : bt->side[bt->branch_of[w] - 1];
    // a multiple of kSlabs blocks, so that every XCD's queue has blocks
    const int64_t want = std::min<int64_t>(b1 - b0, (int64_t)std::max(1, bt->ctx->num_cus) * bt->params.blocks_per_cu);
    const unsigned grid = (unsigned)(std::max<int64_t>(1, (want + kSlabs - 1) / kSlabs) * kSlabs);
    const XQueues q = bt->xq[w];
#define PG_BE(WW) hipLaunchKernelGGL((k_batch_estimate<WW>), dim3(grid), dim3(kBlock), 0, ws, ev, q)
    switch (w) {
      case 1: PG_BE(1); break;
      case 2: PG_BE(2); break;
      case 3: PG_BE(3); break;
      case 4: PG_BE(4); break;
      case 5: PG_BE(5); break;
      case 6: PG_BE(6); break;
      case 7: PG_BE(7); break;
      case 8: PG_BE(8); break;
      case 9: PG_BE(9); break;
      case 10: PG_BE(10); break;
      case 11: PG_BE(11); break;
      case 12: PG_BE(12); break;
      case 13: PG_BE(13); break;
      case 14: PG_BE(14); break;
      case 15: PG_BE(15); break;
      default: PG_BE(16); break;
    }
#undef PG_BE
    PG_LAUNCH_CHECK();
  }
  for (int i = 0; i < kBranches - 1; ++i) {
    PG_HIP(hipEventRecord(bt->join[i], bt->side[i]));
    PG_HIP(hipStreamWaitEvent(s, bt->join[i], 0));
  }
  hipLaunchKernelGGL(k_batch_tc, dim3((unsigned)bt->count), dim3(kBlock), 0, s, (const GraphDesc*)bt->gd,
                     (const double*)bt->Splus, bt->tc);
  PG_LAUNCH_CHECK();
  return PG_OK;
}

void drop_graph(pg_batch* bt) {
  if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
  if (bt->graph) (void)hipGraphDestroy(bt->graph);
  bt->exec = nullptr;
  bt->graph = nullptr;
}

void free_batch(pg_batch* bt) {
  drop_graph(bt);
  for (int i = 0; i < kBranches - 1; ++i) {
    if (bt->side[i]) (void)hipStreamSynchronize(bt->side[i]);
    if (bt->side[i]) (void)hipStreamDestroy(bt->side[i]);
    if (bt->join[i]) (void)hipEventDestroy(bt->join[i]);
  }
  if (bt->fork) (void)hipEventDestroy(bt->fork);
  pfree(bt->gd);
  pfree(bt->items);
  pfree(bt->eitems);
  pfree(bt->off);
  pfree(bt->adj);
  pfree(bt->words);
  pfree(bt->pc);
  pfree(bt->ha);
  pfree(bt->hc);
  pfree(bt->tables);
  pfree(bt->S);
  pfree(bt->Splus);
  pfree(bt->cc);
  pfree(bt->tc);
  pfree(bt->counters);
  delete bt;
}

bool bf_estimator(int est) { return est == PG_EST_BF_AND || est == PG_EST_BF_L || est == PG_EST_BF_PAPAPETROU; }

}  // namespace
}  // namespace pg

using namespace pg;

extern "C" {

int pg_batch_create(pg_ctx* ctx, int32_t count, const int32_t* const* offsets, const int32_t* const* adj,
                    const int32_t* n, const int64_t* nnz, const uint32_t* bits, uint32_t b, uint64_t seed,
                    pg_batch** out) {
  clear_error();
  if (!ctx || !out || count < 1 || !offsets || !adj || !n || !nnz || !bits) return fail(PG_E_INVALID, "bad argument");
  *out = nullptr;
  if (b < 1 || b > 16) return fail(PG_E_INVALID, "b must be in [1, 16]");
  // host checks: bounds, sortedness, no self-loops, symmetry
  int64_t N = 0, A = 0, words = 0, tab = 0;
  for (int32_t g = 0; g < count; ++g) {
    if (n[g] < 0 || nnz[g] < 0 || bits[g] < 64 || bits[g] > 64u * kMaxW || bits[g] % 64)
      return fail(PG_E_INVALID, "graph " + std::to_string(g) + ": bad n, nnz or filter size");
    if (!offsets[g] || (nnz[g] > 0 && !adj[g])) return fail(PG_E_INVALID, "NULL graph array");
    const int32_t* o = offsets[g];
    const int32_t* a = adj[g];
    if (o[0] != 0 || (int64_t)o[n[g]] != nnz[g]) return fail(PG_E_GRAPH, "graph " + std::to_string(g) + ": offsets");
    for (int32_t v = 0; v < n[g]; ++v) {
      if (o[v + 1] < o[v]) return fail(PG_E_GRAPH, "graph " + std::to_string(g) + ": offsets not monotone");
      for (int32_t p = o[v]; p < o[v + 1]; ++p) {
        const int32_t u = a[p];
        if (u < 0 || u >= n[g] || u == v || (p > o[v] && a[p - 1] >= u))
          return fail(PG_E_GRAPH, "graph " + std::to_string(g) + ": bad neighbour list");
        if (!std::binary_search(a + o[u], a + o[u + 1], v))
          return fail(PG_E_GRAPH, "graph " + std::to_string(g) + ": not symmetric");
      }
    }
    N += n[g];
    A += nnz[g];
    words += (int64_t)n[g] * (bits[g] / 64);
    tab += bits[g] + 1;
  }
  PG_HIP(hipSetDevice(ctx->device));
  pg_batch* bt = new (std::nothrow) pg_batch();
  if (!bt) return fail(PG_E_NOMEM, "host allocation failed");
  bt->ctx = ctx;
  bt->count = count;
  bt->N = N;
  bt->arcs = A;
  bt->b = b;
  bt->seed = seed;
  bt->h_gd.resize(count);
  bt->h_off.assign((size_t)N + 1, 0);
  std::vector<int32_t> h_adj((size_t)std::max<int64_t>(A, 1));
  int64_t vb = 0, ab = 0, wb = 0, tb = 0;
  for (int32_t g = 0; g < count; ++g) {
    GraphDesc& d = bt->h_gd[g];
    d.vbase = vb;
    d.wbase = wb;
    d.tbase = tb;
    d.n = n[g];
    d.B = bits[g];
    d.W = bits[g] / 64;
    d.pad = 0;
    for (int32_t v = 0; v <= n[g]; ++v) bt->h_off[vb + v] = ab + offsets[g][v];
    std::copy(adj[g], adj[g] + nnz[g], h_adj.begin() + ab);
    vb += n[g];
    ab += nnz[g];
    wb += (int64_t)n[g] * d.W;
    tb += bits[g] + 1;
  }
  uint64_t ha[16], hc[16];
  hash_constants(PG_BF, seed, b, ha, hc);
  int rc = PG_OK;
  auto P = [&](void** p, size_t bytes) {
    if (rc == PG_OK) rc = palloc(p, std::max<size_t>(bytes, 8));
  };
  P((void**)&bt->gd, sizeof(GraphDesc) * count);
  P((void**)&bt->off, sizeof(int64_t) * (N + 1));
  P((void**)&bt->adj, sizeof(int32_t) * A);
  P((void**)&bt->words, sizeof(uint64_t) * (words + kBfSlackWords));  // team readers may read past the last row
  P((void**)&bt->pc, sizeof(uint32_t) * N);
  P((void**)&bt->ha, sizeof(uint64_t) * b);
  P((void**)&bt->hc, sizeof(uint64_t) * b);
  P((void**)&bt->tables, sizeof(double) * tab);
  P((void**)&bt->S, sizeof(double) * N);
  P((void**)&bt->Splus, sizeof(double) * N);
  P((void**)&bt->cc, sizeof(float) * N);
  P((void**)&bt->tc, sizeof(double) * count);
  P((void**)&bt->counters, sizeof(uint32_t) * kCounters);
  if (rc == PG_OK) {
    hipError_t e = hipMemcpy(bt->gd, bt->h_gd.data(), sizeof(GraphDesc) * count, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(bt->off, bt->h_off.data(), sizeof(int64_t) * (N + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess && A > 0) e = hipMemcpy(bt->adj, h_adj.data(), sizeof(int32_t) * A, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(bt->ha, ha, sizeof(uint64_t) * b, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(bt->hc, hc, sizeof(uint64_t) * b, hipMemcpyHostToDevice);
    if (e != hipSuccess) rc = fail(PG_E_DEVICE, std::string("batch upload: ") + hipGetErrorString(e));
  }
  for (int i = 0; i < kBranches - 1 && rc == PG_OK; ++i) {
    if (hipStreamCreateWithFlags(&bt->side[i], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&bt->join[i], hipEventDisableTiming) != hipSuccess)
      rc = fail(PG_E_DEVICE, "batch streams");
  }
  if (rc == PG_OK && hipEventCreateWithFlags(&bt->fork, hipEventDisableTiming) != hipSuccess)
    rc = fail(PG_E_DEVICE, "batch events");
  if (rc == PG_OK) rc = build_items(bt);
  if (rc != PG_OK) {
    free_batch(bt);
    return rc;
  }
  *out = bt;
  return PG_OK;
}

int pg_batch_set_params(pg_batch* bt, const pg_batch_params* params) {
  clear_error();
  if (!bt || !params) return fail(PG_E_INVALID, "NULL argument");
  pg_batch_params p = *params;
  if (p.tile_vertices == 0) p.tile_vertices = 64;
  if (p.blocks_per_cu == 0) p.blocks_per_cu = 4;
  if (p.tile_vertices < kGroups || p.tile_vertices % kGroups || p.tile_vertices > 4096)
    return fail(PG_E_INVALID, "tile_vertices must be a multiple of 32 in [32, 4096]");
  if (p.blocks_per_cu < 1 || p.blocks_per_cu > 32) return fail(PG_E_INVALID, "blocks_per_cu must be in [1, 32]");
  PG_HIP(hipSetDevice(bt->ctx->device));
  PG_HIP(hipDeviceSynchronize());  // a previous run may still read the work list
  const bool retile = p.tile_vertices != bt->params.tile_vertices;
  bt->params = p;
  drop_graph(bt);
  if (retile) PG_TRY(build_items(bt));
  return PG_OK;
}

int pg_batch_get_params(const pg_batch* bt, pg_batch_params* out) {
  clear_error();
  if (!bt || !out) return fail(PG_E_INVALID, "NULL argument");
  *out = bt->params;
  return PG_OK;
}

int pg_batch_run(pg_batch* bt, int estimator, void* stream) {
  clear_error();
  if (!bt) return fail(PG_E_INVALID, "NULL argument");
  if (!bf_estimator(estimator)) return fail(PG_E_INVALID, "batches use the AND, L or Papapetrou estimator");
  PG_HIP(hipSetDevice(bt->ctx->device));
  return enqueue_run(bt, estimator, (hipStream_t)stream);
}

int pg_batch_capture(pg_batch* bt, int estimator, void* stream) {
  clear_error();
  if (!bt) return fail(PG_E_INVALID, "NULL argument");
  if (!bf_estimator(estimator)) return fail(PG_E_INVALID, "batches use the AND, L or Papapetrou estimator");
  PG_HIP(hipSetDevice(bt->ctx->device));
  hipStream_t s = (hipStream_t)stream;
  if (!s) return fail(PG_E_INVALID, "capture needs an explicit (non-default) stream");
  drop_graph(bt);
  PG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  const int rc = enqueue_run(bt, estimator, s);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (rc != PG_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(PG_E_DEVICE, std::string("end capture: ") + hipGetErrorString(e));
  bt->graph = g;
  PG_HIP(hipGraphInstantiate(&bt->exec, g, nullptr, nullptr, 0));
  return PG_OK;
}

int pg_batch_replay(pg_batch* bt, void* stream) {
  clear_error();
  if (!bt) return fail(PG_E_INVALID, "NULL argument");
  if (!bt->exec) return fail(PG_E_INVALID, "no captured run");
  PG_HIP(hipSetDevice(bt->ctx->device));
  ProfScope ps((hipStream_t)stream, "batch_replay");
  PG_HIP(hipGraphLaunch(bt->exec, (hipStream_t)stream));
  return PG_OK;
}

int pg_batch_results(pg_batch* bt, double* tc, float* cc, void* stream) {
  clear_error();
  if (!bt) return fail(PG_E_INVALID, "NULL argument");
  PG_HIP(hipSetDevice(bt->ctx->device));
  hipStream_t s = (hipStream_t)stream;
  if (tc) PG_HIP(hipMemcpyAsync(tc, bt->tc, sizeof(double) * bt->count, hipMemcpyDeviceToHost, s));
  if (cc) PG_HIP(hipMemcpyAsync(cc, bt->cc, sizeof(float) * bt->N, hipMemcpyDeviceToHost, s));
  PG_HIP(hipStreamSynchronize(s));
  return PG_OK;
}

int pg_batch_autotune(pg_batch* bt, int estimator, void* stream, double* best_ms) {
  clear_error();
  if (!bt) return fail(PG_E_INVALID, "NULL argument");
  if (!bf_estimator(estimator)) return fail(PG_E_INVALID, "batches use the AND, L or Papapetrou estimator");
  PG_HIP(hipSetDevice(bt->ctx->device));
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  PG_HIP(hipEventCreate(&e0));
  PG_HIP(hipEventCreate(&e1));
  pg_batch_params best = bt->params;
  double best_t = 1e300;
  int rc = PG_OK;
  for (int32_t tile : {32, 64, 128, 256}) {
    for (int32_t bpc : {2, 4, 8}) {
      pg_batch_params p{tile, bpc};
      rc = pg_batch_set_params(bt, &p);
      if (rc != PG_OK) break;
      std::vector<float> times;
      for (int rep = 0; rep < 4 && rc == PG_OK; ++rep) {
        hipError_t e = hipEventRecord(e0, s);
        if (e == hipSuccess) rc = enqueue_run(bt, estimator, s);
        if (rc == PG_OK) {
          e = hipEventRecord(e1, s);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float ms = 0.0f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          if (e != hipSuccess) rc = fail(PG_E_DEVICE, std::string("autotune timing: ") + hipGetErrorString(e));
          if (rep > 0) times.push_back(ms);  // the first run warms up
        }
      }
      if (rc != PG_OK) break;
      std::sort(times.begin(), times.end());
      const double med = times[times.size() / 2];
      if (med < best_t) {
        best_t = med;
        best = p;
      }
    }
    if (rc != PG_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != PG_OK) return rc;
  PG_TRY(pg_batch_set_params(bt, &best));
  if (best_ms) *best_ms = best_t;
  return PG_OK;
}

int pg_batch_destroy(pg_batch* bt) {
  clear_error();
  if (!bt) return fail(PG_E_INVALID, "NULL argument");
  PG_HIP(hipSetDevice(bt->ctx->device));
  PG_HIP(hipDeviceSynchronize());
  free_batch(bt);
  return PG_OK;
}

}  // extern "C"
