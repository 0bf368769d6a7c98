// Internal declarations of the ProbGraph GPU library: handle layouts, error
// plumbing and the host-side launchers each .hip file provides.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "probgraph.h"

namespace pg {

// ---- errors ----------------------------------------------------------------
void set_error(const std::string& msg);
void clear_error();
int fail(int code, const std::string& msg);

#define PG_HIP(call)                                                                              \
  do {                                                                                            \
    hipError_t pg_e_ = (call);                                                                    \
    if (pg_e_ != hipSuccess)                                                                      \
      return ::pg::fail(PG_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(pg_e_));      \
  } while (0)

#define PG_TRY(call)                   \
  do {                                 \
    int pg_rc_ = (call);               \
    if (pg_rc_ != PG_OK) return pg_rc_; \
  } while (0)

// Launch-error check right after a kernel launch.
#define PG_LAUNCH_CHECK() PG_HIP(hipGetLastError())

int dmalloc(void** p, size_t bytes, hipStream_t s);  // stream-ordered temporary device allocation
int dfree(void* p, hipStream_t s);
int palloc(void** p, size_t bytes);                 // long-lived device allocation
int pfree(void* p);

// ---- per-kernel device timing ---------------------------------------------------
// While profiling is enabled, a ProfScope records a HIP event on its stream at
// construction and another at destruction; pg_profile_read sums the elapsed
// times per name.
bool prof_enabled();
struct ProfScope {
  ProfScope(hipStream_t s, const char* name);
  ~ProfScope();
  hipStream_t s_;
  const char* name_;
  hipEvent_t start_ = nullptr;
};

// ---- degree bins -----------------------------------------------------------
// Vertices are partitioned once per graph by degree; per-vertex kernels map a
// group of G lanes to one vertex, G growing with the bin.
constexpr int kNumBins = 4;
constexpr int32_t kBinMaxDeg[kNumBins - 1] = {16, 256, 4096};  // bin 3: d > 4096
constexpr int kBinGroup[kNumBins] = {4, 16, 64, 256};

// ---- vertex work plans -----------------------------------------------------
// A plan splits per-vertex work over N_v into three tiers launched together,
// heaviest first:
//   heavy  (d_v >  kMediumMax): chunks of kHeavyChunk arcs, one block each
//   medium (kLightMax < d_v <= kMediumMax): one wave per vertex
//   light  (d_v <= kLightMax): kLightGroup lanes per vertex in the filter
//          build (the clustering kernels pick their own group size)
// (Measured on R-MAT s20, BF-320: light limits of 32 / 64 / 128 / 256 / 512
// vertices gave the build 72 / 54 / 52 / 46 / 46 us, 43 us with 8 loads per
// lane and pass; the triangle count's slab items do best at 256.)
// Isolated vertices stay in the light tier (their sketch rows still have to
// be written; they end the light list). The light list is sorted by
// descending passes of the filter build, ceil(d_v / (kLightGroup *
// kLightUnroll)), in ID order within a pass count: the groups of a wave take
// equally many passes and neighbouring groups keep nearby IDs.
constexpr int32_t kLightMax = 512;
constexpr int32_t kMediumMax = 2048;
constexpr int64_t kHeavyChunk = 2048;
constexpr int kLightGroup = 4;
constexpr int kLightUnroll = 8;  // arcs each lane of a light group loads per pass of the filter build

struct VertexPlan {
  int64_t n_light = 0;
  int32_t* light = nullptr;       // [n_light] light vertices, by descending degree
  int64_t n_empty = 0;            // vertices without arcs: the last n_empty of the light list
  int64_t n_medium = 0;
  int32_t* medium = nullptr;      // [n_medium] medium vertices, ascending
  int64_t n_chunks = 0;
  int32_t* chunk_vertex = nullptr;  // [n_chunks]
  int64_t* chunk_begin = nullptr;   // [n_chunks] arc range of the chunk
  int64_t* chunk_end = nullptr;     // [n_chunks]
  int32_t* chunk_slot = nullptr;    // [n_chunks] index of the chunk's heavy vertex
  int64_t n_heavy = 0;
  int32_t* heavy_first = nullptr;   // [n_heavy + 1] chunks of heavy vertex h: [heavy_first[h], heavy_first[h+1])
  int32_t* sorted = nullptr;        // [n] vertices by tier (backing store of `light` and `medium`)
};

// Plan view passed to kernels by value.
struct PlanView {
  int64_t n_chunks;
  int64_t n_medium;
  int64_t n_medium_blocks;
  int64_t n_light;
  const int32_t* light;
  const int32_t* medium;
  const int32_t* chunk_vertex;
  const int64_t* chunk_begin;
  const int64_t* chunk_end;
  const int32_t* chunk_slot;
  const int32_t* heavy_first;
};

inline PlanView plan_view(const VertexPlan& p) {
  PlanView v;
  v.n_chunks = p.n_chunks;
  v.n_medium = p.n_medium;
  v.n_medium_blocks = (p.n_medium + 3) / 4;
  v.n_light = p.n_light;
  v.light = p.light;
  v.medium = p.medium;
  v.chunk_vertex = p.chunk_vertex;
  v.chunk_begin = p.chunk_begin;
  v.chunk_end = p.chunk_end;
  v.chunk_slot = p.chunk_slot;
  v.heavy_first = p.heavy_first;
  return v;
}

// Blocks of 256 threads a plan launch needs.
inline int64_t plan_blocks(const VertexPlan& p) {
  return p.n_chunks + (p.n_medium + 3) / 4 + (p.n_light * kLightGroup + 255) / 256;
}

// ---- XCD slabs of the triangle count ----------------------------------------
// gfx950 has 8 accelerator dies (XCDs), each with its own 4 MB L2, and hands
// workgroup i of a launch to XCD i mod 8. The vertex IDs are cut into kSlabs
// ranges; block i of the slab part of the triangle-count launch only gathers
// Bloom-filter rows of slab i mod kSlabs, so each L2 caches an eighth of the
// rows instead of all of them.
//
// Only vertices with more than kSliceMin upper neighbours are sliced: item
// (x, v) is v's upper neighbours inside slab x, tiered by their number like a
// VertexPlan but with its own light limit, kSlabLightMax (light items get
// kSlabLightGroup lanes, medium ones a wave, heavy ones chunks of kHeavyChunk
// arcs). The slabs hold about equal numbers of
// these arcs. The remaining vertices ("whole" vertices, 1..kSliceMin upper
// neighbours) are not worth a slab each: their blocks follow the slab blocks,
// kWholeGroup lanes per vertex over all upper neighbours. Light lists are
// sorted by descending arc count, so the groups of a wave walk about equally
// many arcs and few load instructions run with idle lanes.
constexpr int kSlabs = 8;
constexpr int32_t kSliceMin = 64;
constexpr int32_t kSlabLightMax = 256;  // light slab items: at most this many arcs (then a wave, then chunks)
constexpr int kSlabLightGroup = 8;
constexpr int kWholeGroup = 8;      // lanes per light vertex of the clustering-coefficient plan
constexpr int kSlabWholeGroup = 4;  // lanes per whole (unsliced) vertex of the triangle-count slab plan
// Sort buckets of the slab plan's lists (see sort_light_list): light items
// by exact arc count, whole vertices by ceil(upper degree / 16).
constexpr int kSlabLightBucket = 1;
constexpr int kSlabWholeBucket = 16;

struct SlabPlan {
  int32_t* split = nullptr;  // [(kSlabs-1) * n]: split[(x-1)*n + v] = first arc of v into slab x >= 1
  int64_t n_light[kSlabs] = {};
  int64_t n_medium[kSlabs] = {};
  int64_t n_chunks[kSlabs] = {};
  int64_t light_at[kSlabs] = {};   // slab x's light items: verts[light_at[x] ..], by descending arc count
  int64_t medium_at[kSlabs] = {};  // slab x's medium items: verts[medium_at[x] ..]
  int64_t chunk_at[kSlabs] = {};   // slab x's chunks: chunk_*[chunk_at[x] ..]
  int64_t slab_grid = 0;           // blocks of the slab part: kSlabs * (blocks of the busiest slab)
  int64_t n_whole = 0;             // whole vertices: verts[whole_at ..], by descending arc count
  int64_t whole_at = 0;
  int32_t* verts = nullptr;
  int32_t* chunk_vertex = nullptr;
  int64_t* chunk_begin = nullptr;
  int64_t* chunk_end = nullptr;
  // clustering-coefficient plans (over all of N_v) only: where each sliced
  // vertex's item sums go
  int64_t n_sliced = 0;           // vertices with more than kSliceMin arcs
  int32_t* rank = nullptr;        // [n] index among the sliced vertices, -1 for the others
  int32_t* chunk_ptr = nullptr;   // [n_sliced + 1] a sliced vertex's chunks in chunk_list
  int32_t* chunk_list = nullptr;  // chunk indices by sliced vertex, in chunk order
};

// Blocks of slab x (block i of the slab part serves slab i mod kSlabs).
__host__ __device__ inline int64_t slab_blocks(const SlabPlan& p, int x) {
  return p.n_chunks[x] + (p.n_medium[x] + 3) / 4 + (p.n_light[x] * kSlabLightGroup + 255) / 256;
}
// Blocks of the whole launch.
inline int64_t slab_plan_blocks(const SlabPlan& p) {
  return p.slab_grid + (p.n_whole * kSlabWholeGroup + 255) / 256;
}

__device__ __forceinline__ int64_t slab_begin(const int32_t* __restrict__ ustart, const int32_t* __restrict__ split,
                                              size_t n, int x, int32_t v) {
  return x == 0 ? ustart[v] : split[(size_t)(x - 1) * n + v];
}
__device__ __forceinline__ int64_t slab_end(const int32_t* __restrict__ off, const int32_t* __restrict__ split,
                                            size_t n, int x, int32_t v) {
  return x == kSlabs - 1 ? off[v + 1] : split[(size_t)x * n + v];
}

}  // namespace pg

struct pg_ctx {
  int device = 0;
  int num_cus = 0;
  double* h_scalar = nullptr;  // pinned host slot for scalar results
  double* scratch = nullptr;   // the device's fixed workspace (pg_tc_noalloc), not owned
  int64_t scratch_doubles = 0;
};

struct pg_graph {
  pg_ctx* ctx = nullptr;
  int32_t n = 0;
  int64_t nnz = 0;
  int64_t m = 0;
  int32_t max_degree = 0;
  uint64_t wedges = 0;         // sum_v C(d_v, 2)
  bool owns_csr = true;
  int32_t* off = nullptr;      // [n+1]
  int32_t* adj = nullptr;      // [nnz]
  int32_t* deg = nullptr;      // [n]
  int32_t* ustart = nullptr;   // [n] position in adj of the first neighbour above v
  int64_t* upoff = nullptr;    // [n+1] first upper-edge index of v (edges in CSR order)
  pg::VertexPlan plan_all;     // work over N_v (sketch builds, clustering coefficient)
  pg::SlabPlan slabs;          // triangle-count plan over XCD slabs (built on first use)
  pg::SlabPlan slabs_all;      // clustering-coefficient plan over XCD slabs, all of N_v (built on first use)
  int32_t* eu = nullptr;       // [m] smaller endpoint of each undirected edge
  int32_t* ev = nullptr;       // [m] larger endpoint
  int32_t* arc_src = nullptr;  // [nnz] source vertex of each arc
  int32_t* bin_verts = nullptr;              // [n] vertices grouped by degree bin, ascending inside a bin
  int64_t bin_start[pg::kNumBins + 1] = {};  // bin j = bin_verts[bin_start[j] .. bin_start[j+1])
  // degree-oriented CSR for the exact node iterator (built on first use)
  int32_t* poff = nullptr;     // [n+1]
  int32_t* padj = nullptr;     // [m]
  int32_t* parc_src = nullptr; // [m]
  // the oriented lists as a graph of their own (off/adj borrow poff/padj; own
  // degrees d+, degree bins and plan_all), built on first use by oriented sketches
  pg_graph* oriented = nullptr;
  int live_sketches = 0;
};

struct pg_sketches {
  pg_graph* g = nullptr;     // the graph: its edges are the pairs of TC and the all-edge calls
  pg_graph* rows = nullptr;  // whose lists the rows sketch: g, or g->oriented (PG_ORIENTED)
  bool oriented = false;
  int kind = 0;
  uint32_t size = 0;   // B or k
  uint32_t b = 1;
  uint32_t W = 0;      // 64-bit words per Bloom-filter row
  uint64_t seed = 0;
  uint64_t* words = nullptr;  // Bloom-filter rows, line-packed (bf_row_offset)
  uint32_t* pc = nullptr;     // [n]    ones per filter
  uint32_t* sig = nullptr;    // [n*k]  MinHash rows
  uint64_t* ha = nullptr;     // device hash multipliers
  uint64_t* hc = nullptr;     // device hash increments
  double* table = nullptr;    // [kBfTables * (B+1)] estimator tables (Bloom filters), one per estimator
  bool empty_rows_zero = false;  // Bloom filters: the rows of vertices without arcs are known to be zero
  uint64_t* scratch = nullptr;    // heavy-chunk partials: Bloom-filter rows (n_chunks * W words) or
                                  // k-hash (key, element) pairs (n_chunks * k keys, then n_chunks * k uint32)
                                  // or 1-hash candidates (n_chunks * k uint32, when k <= kHeavyChunk)
};

namespace pg {

// ---- launchers (pg_graph.hip) ------------------------------------------------
int graph_prepare(pg_graph* g, bool validate, hipStream_t s);
int graph_arc_sources(pg_graph* g, hipStream_t s);
int graph_orient(pg_graph* g, hipStream_t s);
int graph_oriented(pg_graph* g, hipStream_t s);  // g->oriented (and the oriented CSR) on first use
int graph_slabs(pg_graph* g, hipStream_t s);
int graph_slabs_all(pg_graph* g, hipStream_t s);
int build_plan(pg_graph* g, pg::VertexPlan* plan, hipStream_t s);
void free_plan(pg::VertexPlan* plan);
void free_slabs(pg::SlabPlan* plan);
int exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t count, hipStream_t s);
int fill_u64(uint64_t* p, uint64_t value, int64_t count, hipStream_t s);
// Fixed-order sum of nchunks partials, divided by `divisor`, into out[0].
// Above kWideMax partials it needs sum_chunks_tiles(nchunks) doubles of
// temporary memory: `tiles` if given, else allocated on the stream.
int64_t sum_chunks_tiles(int64_t nchunks);
int sum_chunks(const double* chunks, int64_t nchunks, double divisor, double* out, hipStream_t s,
               double* tiles = nullptr);
int sum_array(const double* x, int64_t count, double divisor, double* out, hipStream_t s);

// ---- launchers (pg_build.hip) ------------------------------------------------
int build_bf(pg_sketches* sk, hipStream_t s);
int build_khash(pg_sketches* sk, hipStream_t s);
int build_onehash(pg_sketches* sk, hipStream_t s);
// Dense row-major copy (n * W words) of line-packed Bloom-filter rows.
int bf_unpack(const pg_sketches* sk, void* rows, hipStream_t s);
// The inverse: line-packed rows from a dense copy, and the popcounts (copied
// from pc, or counted from the rows when pc is NULL).
int bf_pack(pg_sketches* sk, const void* rows, const uint32_t* pc, hipStream_t s);

// ---- launchers (pg_estimate.hip) ---------------------------------------------
// Bloom-filter sets hold one table of B+1 entries per estimator
// (PG_EST_BF_AND .. PG_EST_BF_PAPAPETROU), all filled when the set is made, so
// calls on different streams never rewrite a table another call reads.
constexpr int kBfTables = 4;
int fill_tables(pg_sketches* sk, hipStream_t s);
// The table of estimator `est` of a Bloom-filter set (NULL for MinHash sets).
const double* bf_table(const pg_sketches* sk, int est);
// Estimator table of a Bloom-filter size into a caller-owned [B+1] array.
int fill_table(double* table, uint32_t B, uint32_t b, int est, hipStream_t s);
// Per pair: est / raw / similarity (PG_SIM_* measure) outputs, each nullable.
int estimate_pairs(const pg_sketches* sk, int est, const int32_t* u, const int32_t* v, int64_t npairs,
                   double* est_out, uint32_t* raw_out, float* sim_out, int measure, hipStream_t s);
// Jarvis-Patrick over the m upper edges: keep[m] (nullable) and |C| into d_kept[0].
int estimate_jp(const pg_sketches* sk, int est, int measure, double tau, uint8_t* keep, unsigned long long* d_kept,
                hipStream_t s);
// Deterministic sum of the estimate over pairs into chunk partials; nchunks_out
// receives the number of partials written to `chunks` (sized by chunk_count()).
int64_t chunk_count(int64_t npairs);
int estimate_sum(const pg_sketches* sk, int est, const int32_t* u, const int32_t* v, int64_t npairs,
                 double* chunks, hipStream_t s);
int estimate_cc(const pg_sketches* sk, int est, float* cc, double* vsum, hipStream_t s);
// TC^ = (1/3) sum over the m edges of the estimate, into d_out[0] (device).
// With a workspace the partial sums live there and the call allocates
// nothing; it then needs the graph's triangle-count plan to exist already
// (PG_E_UNSUPPORTED otherwise, or when the partials exceed the workspace).
struct TcWorkspace {
  double* ptr;      // device
  int64_t doubles;  // capacity
};
int estimate_tc(const pg_sketches* sk, int est, double* d_out, hipStream_t s, const TcWorkspace* ws = nullptr);
// The library's fixed workspace on `device` (see pg_tc_noalloc): its device
// address, looked up once per device, and its size.
int noalloc_scratch(int device, double** ptr, int64_t* doubles);

// ---- launchers (pg_exact.hip) ------------------------------------------------
int exact_pairs(const pg_graph* g, int algo, const int32_t* u, const int32_t* v, int64_t npairs,
                uint32_t* out, hipStream_t s);
int exact_tc(pg_graph* g, int algo, uint64_t* d_tc, hipStream_t s);
int exact_cc(pg_graph* g, float* cc, hipStream_t s);
int exact_similarity(const pg_graph* g, int measure, const int32_t* u, const int32_t* v, int64_t npairs, float* out,
                     hipStream_t s);
int exact_jp(const pg_graph* g, int algo, int measure, double tau, uint8_t* keep, unsigned long long* d_kept,
             hipStream_t s);

// ---- launchers (pg_clique.hip) -----------------------------------------------
// 4-clique count into d_count[0]: exact (sk NULL) or from Bloom filters of N+.
int four_cliques(pg_graph* g, const pg_sketches* sk, unsigned long long* d_count, hipStream_t s);
// 4-clique estimate from the AND / OR of the filter of N+_w and a filter of C3,
// FP64 into d_out[0] (device); sk holds Bloom filters of the oriented sets.
int four_cliques_estimate(const pg_sketches* sk, int est, double* d_out, hipStream_t s);

// ---- launchers (pg_cluster.hip) ----------------------------------------------
// Connected components of the kept upper edges (keep NULL: all); label[v] =
// smallest vertex ID of v's component; the component count into d_count[0].
int clusters(const pg_graph* g, const uint8_t* keep, int32_t* label, unsigned long long* d_count, hipStream_t s);

// ---- host utilities (pg_api.hip) ---------------------------------------------
uint64_t splitmix64(uint64_t key, uint64_t i);
void hash_constants(int kind, uint64_t seed, uint32_t count, uint64_t* a, uint64_t* c);

inline unsigned grid_for(int64_t threads, int block, int64_t cap = 1 << 20) {
  int64_t g = (threads + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace pg
