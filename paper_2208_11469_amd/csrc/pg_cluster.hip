// Clusters of a Jarvis-Patrick clustering (Listing "lst:cl"): the connected
// components of (V, C), C a subset of the m upper edges, each vertex labelled
// with the smallest vertex ID of its component.
//
// Lock-free union-find over the edges (the concurrent union-find of
// Jaiganesh and Burtscher, "A high-performance connected components
// implementation for GPUs", HPDC 2018, in its hook-to-smaller form). The
// caller's label array holds the parent pointers. Every pointer ever written
// goes to a smaller ID (initially parent[x] = x; a hook sets parent[b] = a for
// roots a < b; path halving sets parent[x] to its grandparent), so a tree's
// root is its smallest vertex and the final labels are unique: they do not
// depend on the order in which edges were joined.
//
// One lane per edge joins the roots of its endpoints: find both roots, hook
// the larger under the smaller with a compare-and-swap, and retry if that root
// was hooked meanwhile. A failed swap means another lane hooked a root, and
// there are at most n - 1 hooks in all, so no lane tries more than n times
// (the loop bound below is that count; the flag it sets is never reached by a
// correct execution). Parent pointers are read and written with agent-scope
// atomics so that every lane, on any XCD, sees the others' hooks.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pg_device.h"
#include "pg_internal.h"

namespace pg {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int32_t uf_load(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void uf_store(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x. Each step moves to a strictly smaller ID, so the walk ends within
// x steps whatever other lanes write meanwhile.
__device__ __forceinline__ int32_t uf_find(int32_t* parent, int32_t x) {
  for (;;) {
    const int32_t p = uf_load(parent + x);
    if (p == x) return x;
    const int32_t gp = uf_load(parent + p);
    if (gp == p) return p;
    uf_store(parent + x, gp);  // path halving: x now skips p
    x = gp;
  }
}

// Root of x without path halving, for the pass after every union is done:
// there the only stores are lanes writing a vertex's final root into its own
// slot, and a halving store from another lane (from a pointer it read before
// that) could overwrite such a root with an inner vertex.
__device__ __forceinline__ int32_t uf_root(const int32_t* parent, int32_t x) {
  for (;;) {
    const int32_t p = uf_load(parent + x);
    if (p == x) return x;
    x = p;
  }
}

__global__ __launch_bounds__(kBlock) void k_uf_init(int32_t* __restrict__ parent, int32_t n) {
  for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock)
    parent[v] = (int32_t)v;
}

__global__ __launch_bounds__(kBlock) void k_uf_union(const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                                                     const uint8_t* __restrict__ keep, int64_t m, int32_t* parent,
                                                     int64_t max_tries, unsigned long long* __restrict__ overflow) {
  for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < m; e += (int64_t)gridDim.x * kBlock) {
    if (keep && !keep[e]) continue;
    int32_t a = eu[e], b = ev[e];
    bool joined = false;
    for (int64_t t = 0; t < max_tries; ++t) {
      a = uf_find(parent, a);
      b = uf_find(parent, b);
      if (a == b) {
        joined = true;
        break;
      }
      if (a > b) {
        const int32_t tmp = a;
        a = b;
        b = tmp;
      }
      int32_t expected = b;
      if (__hip_atomic_compare_exchange_strong(parent + b, &expected, a, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT)) {
        joined = true;
        break;
      }
    }
    if (!joined) atomicOr(overflow, 1ull);
  }
}

// label[v] = root of v; the roots are counted (one integer atomic per block).
__global__ __launch_bounds__(kBlock) void k_uf_flatten(int32_t* parent, int32_t n,
                                                       unsigned long long* __restrict__ count) {
  __shared__ uint32_t roots;
  if (threadIdx.x == 0) roots = 0;
  __syncthreads();
  uint32_t mine = 0;
  for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
    const int32_t r = uf_root(parent, (int32_t)v);
    uf_store(parent + v, r);
    mine += r == (int32_t)v ? 1u : 0u;
  }
  if (mine) atomicAdd(&roots, mine);
  __syncthreads();
  if (threadIdx.x == 0 && roots) atomicAdd(count, (unsigned long long)roots);
}

}  // namespace

// d_count[0] receives the number of components, d_count[1] is nonzero if a
// union ran out of tries (never in a correct execution).
int clusters(const pg_graph* g, const uint8_t* keep, int32_t* label, unsigned long long* d_count, hipStream_t s) {
  PG_TRY(fill_u64((uint64_t*)d_count, 0, 2, s));
  if (g->n <= 0) return PG_OK;
  ProfScope ps(s, "clusters");
  hipLaunchKernelGGL(k_uf_init, dim3(grid_for(g->n, kBlock, 65536)), dim3(kBlock), 0, s, label, g->n);
  PG_LAUNCH_CHECK();
  if (g->m > 0) {
    hipLaunchKernelGGL(k_uf_union, dim3(grid_for(g->m, kBlock, 65536)), dim3(kBlock), 0, s, g->eu, g->ev, keep, g->m,
                       label, (int64_t)g->n + 1, d_count + 1);
    PG_LAUNCH_CHECK();
  }
  // a few blocks per CU: each block adds its root count to one shared counter
  const unsigned flat_grid = grid_for(g->n, kBlock, (int64_t)std::max(1, g->ctx->num_cus) * 8);
  hipLaunchKernelGGL(k_uf_flatten, dim3(flat_grid), dim3(kBlock), 0, s, label, g->n, d_count);
  PG_LAUNCH_CHECK();
  return PG_OK;
}

}  // namespace pg
