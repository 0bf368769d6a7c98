/*
 * probgraph.h -- C ABI of the ProbGraph GPU library (MI355X / gfx950).
 *
 * ProbGraph (Besta et al., SC22) replaces the exact neighbourhood
 * intersections |N_u cap N_v| of graph-mining kernels by estimates computed
 * from fixed-size per-vertex sketches (Section 5, usage example Listing
 * "lst:example"): the caller (1) builds probabilistic representations of all
 * neighbourhoods -- Bloom filters, k-hash or 1-hash MinHash -- and (2) asks
 * for intersection estimates, from which triangle count, clustering
 * coefficients and Jaccard similarities follow.
 *
 * Conventions for every call below:
 *   - Pure C99 interface: only <stdint.h>/<stddef.h> types and opaque handles.
 *   - Return value: PG_OK (0) or a negative PG_E_* code; no call throws or
 *     aborts. pg_last_error() returns a thread-local description of the last
 *     failure on the calling thread.
 *   - Pointers to arrays are DEVICE pointers (memory of the context's GPU)
 *     unless the description says "host". Output buffers are owned and
 *     allocated by the caller; handles are owned by the library and freed by
 *     their *_destroy call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the legacy default
 *     stream). Calls enqueue their work on it and return without waiting,
 *     except calls that return a scalar through a host pointer, which wait for
 *     the stream before returning.
 *   - A pg_ctx and the handles made from it may be used by one host thread at
 *     a time; separate contexts are independent.
 *   - Work plans of a graph (the XCD slab plans of the triangle count and of
 *     the clustering coefficient) are built and allocated by the first call
 *     that needs them and kept with the graph; per-call temporaries come from
 *     the device's stream-ordered pool (pg_ctx_create lets it keep up to
 *     1 GiB of freed memory for reuse).
 *   - Vertex IDs are int32 in [0, n). Graphs are undirected CSR: offsets[n+1]
 *     and adj[nnz], each N_v = adj[offsets[v] .. offsets[v+1]) sorted
 *     ascending, symmetric, with no duplicates and no self-loops (Section 2.1).
 */
#ifndef PROBGRAPH_H
#define PROBGRAPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes -------------------------------------------------------- */
#define PG_OK 0
#define PG_E_INVALID (-1)     /* bad argument: NULL, range, size, kind/estimator mismatch */
#define PG_E_GRAPH (-2)       /* CSR rejected by PG_VALIDATE (unsorted, duplicate, self-loop, asymmetric, out of range) */
#define PG_E_NOMEM (-3)       /* device or host allocation failed */
#define PG_E_DEVICE (-4)      /* a HIP runtime call failed */
#define PG_E_UNSUPPORTED (-5) /* valid request the library does not serve (a size beyond an on-chip buffer, ...) */
#define PG_E_BUSY (-6)        /* serving: request not admitted yet (no slot or memory) */

/* ---- sketch kinds (Section 2.4) ----------------------------------------- */
#define PG_BF 1        /* Bloom filter of B bits with b hash functions */
#define PG_MH_KHASH 2  /* k-hash MinHash: k minima of k hash functions */
#define PG_MH_1HASH 3  /* 1-hash MinHash: k smallest elements under one hash */
/* Flag OR-ed into the kind of pg_build_sketches: sketch the degree-oriented
 * sets N+_v = {u in N_v : R(v) < R(u)}, R = (degree, ID) ascending (Listing
 * "lst:tc"), instead of N_v. */
#define PG_ORIENTED 256 /* bit 8 */

/* ---- estimators of |X cap Y| --------------------------------------------- */
#define PG_EST_BF_AND 1           /* -(B/b) ln(1 - c~/B), c = ones(B_X AND B_Y): Eq. "bf_int", divergence fix of Appendix C */
#define PG_EST_BF_L 2             /* c / b: Eq. "limit_xs" */
#define PG_EST_BF_OR 3            /* |X| + |Y| + (B/b) ln(1 - c~_or/B), c_or = ones(B_X OR B_Y): Eq. "bf_int_union" */
#define PG_EST_BF_PAPAPETROU 4    /* ln(1 - c~/B) / (b ln(1 - 1/B)) on the AND (Section 8.1) */
#define PG_EST_MH_KHASH 5         /* s = #positions i with M_X[i] = M_Y[i]; J = s/k; I = J/(1+J)(|X|+|Y|): Eq. "est_int_mh" */
#define PG_EST_MH_1HASH 6         /* s = |U cap M_X cap M_Y|, U = bottom-k' of M_X u M_Y, k' = min(k, |M_X u M_Y|); J = s/k' (Section 4.4) */
#define PG_EST_MH_1HASH_LITERAL 7 /* s = |M_X cap M_Y|, J = s/k (Section 4.4, as printed) */
/* KMV (Section "Beyond Bloom Filter and MinHash") on 1-hash rows: the KMV of X
 * is the hashes h(x) = ((key(x) >> 11) + 1) * 2^-53 of the row's elements (the
 * k smallest keys of X). K_{X u Y} = the k smallest of K_X u K_Y, and
 * |X u Y|^ = (k - 1) / max K_{X u Y}; when both rows hold fewer than k values
 * they hold the whole sets and the union is counted. An empty set gives 0. */
#define PG_EST_KMV 8              /* |X| + |Y| - |X u Y|^, exact sizes: Eq. "est_inter_set_kmv_exactsets" */
#define PG_EST_KMV_SKETCH_SIZES 9 /* |X|^ + |Y|^ - |X u Y|^, |X|^ = (k - 1) / max K_X (or the count below k): Eq. "est_inter_set_kmv" */

/* ---- graph flags -------------------------------------------------------- */
#define PG_MEM_HOST 0u   /* offsets/adj are host pointers (copied to the device) */
#define PG_MEM_DEVICE 1u /* offsets/adj are device pointers */
#define PG_BORROW 2u     /* with PG_MEM_DEVICE: use the caller's arrays in place; they must outlive the graph */
#define PG_VALIDATE 4u   /* check the CSR invariants on the device; PG_E_GRAPH if violated */

/* ---- exact baselines ---------------------------------------------------- */
#define PG_EXACT_MERGE 1  /* sorted-list intersection: binary search of the shorter list in the longer (Fig. 1, Table "tab:queries-int") */
#define PG_EXACT_BITMAP 2 /* per-vertex bitmap of N_v in on-chip memory, probed by the other list */

typedef struct pg_ctx pg_ctx;
typedef struct pg_graph pg_graph;
typedef struct pg_sketches pg_sketches;

typedef struct pg_graph_info {
  int32_t n;          /* vertices */
  int32_t max_degree; /* d */
  int64_t nnz;        /* arcs = 2m */
  int64_t m;          /* undirected edges */
} pg_graph_info;

typedef struct pg_sketch_info {
  int32_t kind;          /* PG_BF, PG_MH_KHASH, PG_MH_1HASH */
  uint32_t size;         /* B (bits) for PG_BF, k for MinHash */
  uint32_t b;            /* hash functions per Bloom filter (1 for MinHash) */
  uint32_t row_bytes;    /* bytes per vertex row: B/8, or 4k */
  uint64_t seed;         /* seed the hash constants were drawn from */
  uint64_t total_bytes;  /* device bytes held (rows + per-vertex popcounts) */
} pg_sketch_info;

/* Thread-local text of the last error ("" if none). Never NULL. */
const char* pg_last_error(void);

/* Library version string. */
const char* pg_version(void);

/* Context on GPU `device`. *out receives the handle. */
int pg_ctx_create(int device, pg_ctx** out);
int pg_ctx_destroy(pg_ctx* ctx);

/* Device-resident CSR graph (Section 2.1) plus the derived arrays every later
 * call uses: degrees and the m undirected edges (v, u), v < u, in CSR order
 * ("upper edges"). With PG_MEM_HOST the arrays are copied; with PG_MEM_DEVICE
 * they are copied unless PG_BORROW. Waits for `stream`. Destroying a graph
 * while sketches built on it are alive fails with PG_E_INVALID. */
int pg_graph_create(pg_ctx* ctx, int32_t n, int64_t nnz, const int32_t* offsets, const int32_t* adj,
                    uint32_t flags, void* stream, pg_graph** out);
int pg_graph_destroy(pg_graph* g);
int pg_graph_get_info(const pg_graph* g, pg_graph_info* out /* host */);
/* Copy the upper edges into eu[m], ev[m] (device). */
int pg_graph_upper_edges(const pg_graph* g, int32_t* eu, int32_t* ev, void* stream);

/* Bloom-filter size for storage budget s in (0, 1] (Section 5.1): the largest
 * multiple of 64 bits B with n*B <= s * 8 * CSR bytes, CSR bytes =
 * 4(n+1) + 4 nnz; at least 64. *bits is a host pointer. */
int pg_sketch_bits_for_budget(const pg_graph* g, double s, uint32_t* bits);

/* Build one sketch per vertex (Section 2.4, construction costs Table
 * "tab:constr").
 *   kind PG_BF:       size = B bits, a multiple of 64 in [64, 4096]; b in [1, 16].
 *   kind PG_MH_KHASH: size = k in [1, 1024]; b ignored.
 *   kind PG_MH_1HASH: size = k in [1, 1024]; b ignored.
 * Hashing (the paper's MurmurHash3 with a time seed is replaced by a seeded,
 * reproducible family):
 *   mix(z)        = SplitMix64's output mix (Steele, Lea, Flood 2014)
 *   sm(key, i)    = mix(key + (i+1) * 0x9E3779B97F4A7C15)
 *   key           = seed XOR tag, tag = 0x42462D48 (PG_BF), 0x4B482D48
 *                   (PG_MH_KHASH), 0x31482D48 (PG_MH_1HASH)
 *   a_i = sm(key, 2i) | 1,  c_i = sm(key, 2i+1),  g_i(x) = a_i*x + c_i mod 2^64
 *   Bloom-filter bit of x: ((g_i(x) >> 32) * B) >> 32, for i < b
 *   MinHash key of x:      mix(g_i(x)) (injective on 64-bit words: no ties)
 * Equal (graph, kind, size, b, seed) give bit-identical sketches. Rows as
 * exported (pg_sketches_export): BF rows of B/64 uint64 words, bit t of the
 * filter = bit (t & 63) of word (t >> 6); MinHash rows of k uint32 vertex IDs
 * (0xFFFFFFFF = empty slot); k-hash slot i holds the argmin of key_i; 1-hash
 * rows hold the min(k, d_v) smallest keys' elements in ascending key order.
 * (Inside the library BF rows are packed so that none crosses a 128-byte
 * line; export returns them dense.)
 * With kind | PG_ORIENTED the rows sketch N+_v (degree order, see
 * PG_ORIENTED) and the estimators take d+_v = |N+_v| as the set sizes. Such a
 * set serves pg_intersect_edges (estimates of |N+_u cap N+_v|), pg_tc (the
 * oriented form below) and pg_sketches_rebuild / export; pg_cc, pg_jaccard,
 * pg_similarity, pg_jarvis_patrick and servers are defined on N_v and return
 * PG_E_UNSUPPORTED for it. pg_sketches_get_info reports kind | PG_ORIENTED. */
int pg_build_sketches(pg_ctx* ctx, const pg_graph* g, int kind, uint32_t size, uint32_t b, uint64_t seed,
                      void* stream, pg_sketches** out);
int pg_sketches_destroy(pg_sketches* sk);
int pg_sketches_get_info(const pg_sketches* sk, pg_sketch_info* out /* host */);
/* Copy the rows (n * row_bytes bytes) and, for PG_BF, the per-vertex
 * popcounts (pc[n]) into caller device buffers; either may be NULL. */
int pg_sketches_export(const pg_sketches* sk, void* rows, uint32_t* pc, void* stream);
/* Checkpoint / resume: a sketch set on graph g from rows exported by
 * pg_sketches_export, without hashing. kind (with PG_ORIENTED if set), size,
 * b and seed are those pg_sketches_get_info reports for the exported set (the
 * seed keeps pg_sketches_rebuild and the 1-hash estimators consistent); rows
 * (device, n * row_bytes, the export layout) and, for PG_BF, pc (device, n;
 * NULL counts the ones of the rows). On the graph the rows were built on, the
 * set is bit-identical to the exported one. */
int pg_sketches_import(pg_ctx* ctx, const pg_graph* g, int kind, uint32_t size, uint32_t b, uint64_t seed,
                       const void* rows, const uint32_t* pc, void* stream, pg_sketches** out);

/* Estimate |N_u cap N_v| for npairs pairs (u[i], v[i]); u = v = NULL means the
 * graph's m upper edges in CSR order (npairs ignored). est (FP64) and raw
 * (the integer count the estimator consumes: c, c_or or s; for the KMV
 * estimators min(k, |M_u u M_v|)) may each be NULL.
 * The estimator must match the sketch kind. */
int pg_intersect_edges(pg_ctx* ctx, const pg_sketches* sk, int estimator, const int32_t* u, const int32_t* v,
                       int64_t npairs, double* est, uint32_t* raw, void* stream);

/* Estimated triangle count TC^ = (1/3) sum over the m edges of the estimate
 * (Section 7). For an oriented sketch set (PG_ORIENTED) TC^ = sum over the m
 * edges of the estimate of |N+_u cap N+_v|, without the 1/3: the node
 * iterator of Listing "lst:tc" counts each triangle once, at its two
 * lowest-ranked vertices, and the intersection is symmetric, so each edge
 * counts once. *tc is a host pointer; waits for `stream`. */
int pg_tc(pg_ctx* ctx, const pg_sketches* sk, int estimator, double* tc, void* stream);

/* Same estimate written to d_tc[0] (device FP64); enqueued on `stream`
 * without waiting, so successive calls pipeline. */
int pg_tc_async(pg_ctx* ctx, const pg_sketches* sk, int estimator, double* d_tc, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the estimate
 * of pg_tc_async, bit-identical to it, written to d_tc[0] (device FP64) and
 * enqueued on `stream` without waiting. The call allocates and frees nothing:
 * its partial sums go to a fixed device workspace of 16 MiB (2^21 FP64
 * values) that the library holds on each GPU from the first pg_ctx_create on
 * that GPU until the process ends. Every call on one GPU shares that workspace
 * and leaves its last partials there; calls in order on one stream are safe,
 * while calls that overlap on one GPU (other streams, other contexts of the
 * same device) race and must be ordered by the caller. Errors: PG_E_INVALID as
 * pg_tc_async; PG_E_UNSUPPORTED if the graph's triangle-count plan does not
 * exist yet (the first pg_tc or pg_tc_async call on a sketch set of the graph
 * builds it, and allocates) or if the partial sums exceed the workspace. */
int pg_tc_noalloc(pg_ctx* ctx, const pg_sketches* sk, int estimator, double* d_tc, void* stream);

/* Estimated local clustering coefficient cc[n] (device, FP32 rounded once
 * from FP64): cc_v = sum_{u in N_v} I^(u,v) / (d_v (d_v - 1)), 0 if d_v < 2.
 * If transitivity (host) is not NULL it receives 3 TC^ / sum_v C(d_v, 2) and
 * the call waits for `stream`. */
int pg_cc(pg_ctx* ctx, const pg_sketches* sk, int estimator, float* cc, double* transitivity, void* stream);

/* Estimated Jaccard similarity per pair (Listing "lst:sim"):
 * J = I_c / (d_u + d_v - I_c), I_c = the estimate clamped to [0, min(d_u, d_v)];
 * 0 when d_u + d_v = 0. u = v = NULL means the m upper edges. out: FP32. */
int pg_jaccard(pg_ctx* ctx, const pg_sketches* sk, int estimator, const int32_t* u, const int32_t* v,
               int64_t npairs, float* out, void* stream);

/* ---- exact baselines on the same graph ---------------------------------- */
/* Exact |N_u cap N_v| per pair (u = v = NULL: the m upper edges, in CSR
 * order). algo PG_EXACT_MERGE: binary search of the shorter list in the longer
 * one, any pair list. PG_EXACT_BITMAP: each vertex's list is marked in an
 * on-chip bitmap and its upper neighbours' lists are probed against it; it
 * serves u = v = NULL only and returns PG_E_UNSUPPORTED for explicit pairs. */
int pg_exact_intersect_edges(pg_ctx* ctx, const pg_graph* g, int algo, const int32_t* u, const int32_t* v,
                             int64_t npairs, uint32_t* out, void* stream);
/* Exact triangle count by the degree-ordered node iterator (Listing
 * "lst:tc"): orient every edge towards the endpoint of larger (degree, ID)
 * and sum |N+_v cap N+_u| over the oriented edges, each intersection by merge
 * (PG_EXACT_MERGE) or by bitmap (PG_EXACT_BITMAP). *tc host; waits. */
int pg_exact_tc(pg_ctx* ctx, const pg_graph* g, int algo, uint64_t* tc, void* stream);
/* Exact local clustering coefficient (FP32) and, optionally, transitivity (host; waits). */
int pg_exact_cc(pg_ctx* ctx, const pg_graph* g, float* cc, double* transitivity, void* stream);
/* Exact Jaccard similarity per pair (FP32); u = v = NULL: the m upper edges. */
int pg_exact_jaccard(pg_ctx* ctx, const pg_graph* g, const int32_t* u, const int32_t* v, int64_t npairs,
                     float* out, void* stream);

/* ---- vertex similarity and Jarvis-Patrick clustering ---------------------- */
/* Similarity of two neighbourhoods A = N_u, B = N_v (Listing "lst:sim"). */
#define PG_SIM_COMMON 0  /* |A cap B| (common neighbours); an estimate is passed on as it is */
#define PG_SIM_JACCARD 1 /* |A cap B| / |A cup B|; 0 when the union is empty */
#define PG_SIM_OVERLAP 2 /* |A cap B| / min(|A|, |B|); 0 when the smaller set is empty */
#define PG_SIM_TOTAL 3   /* |A cup B| = |A| + |B| - |A cap B| (total neighbours) */

/* Estimated similarity per pair, FP32 rounded once from FP64. For Jaccard,
 * overlap and total neighbours the intersection estimate is first clamped to
 * [0, min(d_u, d_v)], the range of a true intersection. u = v = NULL: the m
 * upper edges in CSR order; pairs with an ID outside [0, n) give NaN. An
 * unknown measure gives PG_E_INVALID. */
int pg_similarity(pg_ctx* ctx, const pg_sketches* sk, int estimator, int measure, const int32_t* u,
                  const int32_t* v, int64_t npairs, float* out, void* stream);
/* Exact similarity per pair (FP32) from exact intersections by merge. */
int pg_exact_similarity(pg_ctx* ctx, const pg_graph* g, int measure, const int32_t* u, const int32_t* v,
                        int64_t npairs, float* out, void* stream);

/* Jarvis-Patrick clustering (Listing "lst:cl"): the clustering C holds the
 * edges whose endpoints' similarity (`measure`, computed from the estimate) is
 * greater than tau; the comparison is made in FP64. keep (device, m bytes,
 * nullable) receives 1 for the upper edges in C and 0 for the others, in CSR
 * upper-edge order; kept (host, nullable) receives |C|, and then the call
 * waits for `stream`. At least one of keep and kept must be given. */
int pg_jarvis_patrick(pg_ctx* ctx, const pg_sketches* sk, int estimator, int measure, double tau, uint8_t* keep,
                      int64_t* kept, void* stream);
/* The same clustering from exact intersections; algo PG_EXACT_MERGE or
 * PG_EXACT_BITMAP (see pg_exact_intersect_edges). Needs m 4-byte words of
 * temporary device memory. */
int pg_exact_jarvis_patrick(pg_ctx* ctx, const pg_graph* g, int algo, int measure, double tau, uint8_t* keep,
                            int64_t* kept, void* stream);

/* Clusters of an edge set C: the connected components of (V, C). label
 * (device, n int32) receives for every vertex the smallest vertex ID of its
 * component, so a vertex with no edge in C labels itself. keep (device, m
 * bytes) selects C among the m upper edges (nonzero = in C); NULL takes every
 * edge of the graph. nclusters (host, nullable) receives the number of
 * components, and then the call waits for `stream`. The labels are unique, so
 * they do not depend on scheduling. */
int pg_clusters(pg_ctx* ctx, const pg_graph* g, const uint8_t* keep, int32_t* label, int64_t* nclusters,
                void* stream);

/* ---- 4-clique counting ----------------------------------------------------- */
/* Reformulated 4-clique count (Listing "lst:fcl"): with the degree order R of
 * the triangle count, for every oriented edge (u, v), C3 = N+_u cap N+_v, and
 * every w in C3 adds |N+_w cap C3|; each 4-clique counts once. *count is a
 * host pointer; the calls wait for `stream`. The triangle lists C3 are held
 * on chip: graphs whose largest oriented degree exceeds 4080 (exact) or 2720
 * (membership queries) give PG_E_UNSUPPORTED. */
/* Exact: |N+_w cap C3| by binary search in N+_w. */
int pg_exact_four_cliques(pg_ctx* ctx, const pg_graph* g, uint64_t* count, void* stream);
/* Estimated: |N+_w cap C3| = the number of x in C3 ranked above w (the only
 * elements N+_w can hold) whose b bits are all set in the Bloom filter of
 * N+_w (membership queries, Section 2.4; false positives only, so the
 * estimate is never below the exact count). sk must hold Bloom filters of the
 * oriented sets (PG_BF | PG_ORIENTED), else PG_E_INVALID. */
int pg_four_cliques(pg_ctx* ctx, const pg_sketches* sk, uint64_t* count, void* stream);
/* Estimated with sketch intersections (the form whose work the paper bounds
 * by B/W word operations per w): for every oriented edge the library builds a
 * Bloom filter of C3 with the hash functions of sk, and |N+_w cap C3| is
 * estimated from it and the filter of N+_w by `estimator`: PG_EST_BF_AND,
 * PG_EST_BF_L or PG_EST_BF_PAPAPETROU (from the ones of the AND, Eqs.
 * "bf_int", "limit_xs" and Section 8.1) or PG_EST_BF_OR (|N+_w| + |C3| and the
 * ones of the OR, Eq. "bf_int_union"). *count (host) receives the FP64 sum
 * over all (edge, w); it does not depend on scheduling. sk must hold Bloom
 * filters of the oriented sets (PG_BF | PG_ORIENTED), else PG_E_INVALID; any
 * other estimator gives PG_E_INVALID. PG_E_UNSUPPORTED when the estimator
 * table (8 (B + 1) bytes) and four C3 buffers (8 W + 4 (d+_max + 1) bytes
 * each, d+_max the largest oriented degree) exceed 128 KiB of LDS. Synchronises
 * `stream`. */
int pg_four_cliques_estimate(pg_ctx* ctx, const pg_sketches* sk, int estimator, double* count, void* stream);

/* Recompute the rows of existing sketches in place (same kind, size and b;
 * new hash constants from `seed`), e.g. after the graph's arrays changed or to
 * draw a fresh sketch set. Allocates nothing. */
int pg_sketches_rebuild(pg_ctx* ctx, pg_sketches* sk, uint64_t seed, void* stream);

/* ---- serving: resident sketches, continuous batching ---------------------- */
/* A server keeps a graph and its sketch sets resident and answers vertex-pair
 * queries (common-neighbour estimates or Jaccard similarities, Listing
 * "lst:sim") as they arrive. The memory budget is a staging arena of pinned
 * host memory that the GPU reads and writes directly, 16 bytes per pair (the
 * two IDs and the answer). A request is admitted if a contiguous range of the
 * arena for its pairs is free; submit writes its pairs there (on the calling
 * thread) and otherwise returns PG_E_BUSY. (The arena is split into up to 16
 * equal parts of at least four largest requests each; a range lies within
 * one part.) Up to max_batches_in_flight batches
 * run concurrently on separate streams; requests submitted while batches run
 * join the next batch as soon as a batch slot frees. A request's range (its
 * bytes of the budget) is released when the request is collected: by
 * pg_server_wait, or by the pg_server_poll that first finds it finished; both
 * copy its answers into its output buffer on the calling thread. Per-pair
 * results do not depend on batching: a request's result is bit-identical alone
 * and in any mix. The graph and sketch sets must outlive the server. Several
 * threads may submit, poll and wait at the same time (each ticket collected by
 * one of them). */
#define PG_OP_CN 1      /* estimate of |N_u cap N_v| (common neighbours), FP64 */
#define PG_OP_JACCARD 2 /* estimated Jaccard similarity, FP32 (rounded once from FP64) */

typedef struct pg_server pg_server;

typedef struct pg_server_params {
  int32_t max_batches_in_flight; /* concurrent batches (streams); 0 = 3 */
  int32_t max_pairs_per_request; /* 0 = 65536 */
  int64_t max_batch_pairs;       /* pairs packed into one launch; 0 = 1 << 20; at most 1 << 30 */
  uint64_t memory_budget_bytes;  /* admission budget; 0 = 256 MiB */
} pg_server_params;

typedef struct pg_request {
  int32_t op;        /* PG_OP_CN or PG_OP_JACCARD */
  int32_t sketch;    /* index into the server's sketch sets */
  int32_t estimator; /* must match that set's kind */
  int32_t reserved;  /* 0 */
  int64_t npairs;    /* 1 .. max_pairs_per_request */
  const int32_t* u;  /* host [npairs]; copied during submit */
  const int32_t* v;  /* host [npairs]; copied during submit */
  void* out;         /* host: double[npairs] (CN) or float[npairs] (Jaccard); written by the server */
} pg_request;

typedef struct pg_server_stats {
  uint64_t submitted;        /* admitted requests */
  uint64_t rejected_busy;    /* PG_E_BUSY answers */
  uint64_t rejected_invalid; /* malformed requests refused before enqueue */
  uint64_t completed;        /* requests whose results were delivered */
  uint64_t batches;          /* launches */
  uint64_t pairs;            /* pairs answered */
  uint64_t max_in_flight;    /* most batches launched and not yet retired at one time */
  uint64_t max_batch_requests; /* most requests packed into one launch */
} pg_server_stats;

/* sketches: host array of nsketches handles built on `g`. params may be NULL. */
int pg_server_create(pg_ctx* ctx, const pg_graph* g, pg_sketches* const* sketches, int32_t nsketches,
                     const pg_server_params* params, pg_server** out);
/* Validates and admits a request (*ticket receives its id, host pointer).
 * PG_E_INVALID: malformed (op, sketch index, estimator/kind mismatch, npairs
 * out of range or above the budget's 16-byte pair slots, a vertex ID outside
 * [0, n)); PG_E_BUSY: not admitted now (no free range of the budget). */
int pg_server_submit(pg_server* srv, const pg_request* req, uint64_t* ticket);
/* *done = 1 once the request's results are in its out buffer: the first poll
 * that finds the request finished copies them there and releases its bytes.
 * The ticket stays valid until pg_server_wait. */
int pg_server_poll(pg_server* srv, uint64_t ticket, int32_t* done);
/* Blocks until the request is answered and its results are in its out buffer,
 * then releases the ticket; latency_ms (host, nullable) receives the time from
 * submit to that point. */
int pg_server_wait(pg_server* srv, uint64_t ticket, double* latency_ms);
int pg_server_get_stats(pg_server* srv, pg_server_stats* out);
/* Load replay: submits reqs[0..nreq) -- at t0 + arrival_s[i] (open loop) or,
 * with arrival_s NULL, in order while at most max_outstanding requests are
 * unanswered (closed loop) -- retrying while the server answers PG_E_BUSY, and
 * writes each request's latency from its arrival to its collected result (host
 * array latency_ms). Up to four threads submit and four collect (request i by
 * thread i mod 4 of each). *elapsed_s (nullable) receives the wall time of the
 * whole replay. */
int pg_server_replay(pg_server* srv, int64_t nreq, const pg_request* reqs, const double* arrival_s,
                     int32_t max_outstanding, double* latency_ms, double* elapsed_s);
/* Waits for every admitted request, stops the engine and frees the server. */
int pg_server_destroy(pg_server* srv);

/* ---- batched small graphs ---------------------------------------------------- */
/* Many independent graphs processed together: per-graph Bloom filters (each
 * graph its own B), then per-graph estimated triangle count and per-vertex
 * clustering coefficient, in persistent launches that pull (graph, vertex tile)
 * work items from a queue ordered by cost. The run allocates nothing and uses
 * no memset, so it can be captured in a HIP graph and replayed. Results do not
 * depend on the tuning parameters or on scheduling. */
typedef struct pg_batch pg_batch;

typedef struct pg_batch_params {
  int32_t tile_vertices;   /* light vertices per work item, a multiple of 32; 0 = 64 */
  int32_t blocks_per_cu;   /* persistent blocks per compute unit; 0 = 4 */
} pg_batch_params;

/* Host CSR arrays of `count` graphs (offsets[i] has n[i]+1 entries, adj[i]
 * nnz[i]); bits[i] = Bloom-filter size of graph i (multiple of 64, <= 1024).
 * The arrays are copied. Graph invariants are checked on the host (bounds
 * always; sortedness and symmetry too). */
int pg_batch_create(pg_ctx* ctx, int32_t count, const int32_t* const* offsets, const int32_t* const* adj,
                    const int32_t* n, const int64_t* nnz, const uint32_t* bits, uint32_t b, uint64_t seed,
                    pg_batch** out);
int pg_batch_set_params(pg_batch* bt, const pg_batch_params* params);
int pg_batch_get_params(const pg_batch* bt, pg_batch_params* out);
/* Enqueue one run: build every filter, estimate every vertex's clustering
 * coefficient and every graph's triangle count with `estimator` (a Bloom-filter
 * estimator). */
int pg_batch_run(pg_batch* bt, int estimator, void* stream);
/* Capture one run (on `stream`) into a HIP graph; pg_batch_replay launches it. */
int pg_batch_capture(pg_batch* bt, int estimator, void* stream);
int pg_batch_replay(pg_batch* bt, void* stream);
/* Results of the last completed run (host arrays; waits for `stream`):
 * tc[count], and cc[sum of n] in graph order (either may be NULL). */
int pg_batch_results(pg_batch* bt, double* tc, float* cc, void* stream);
/* Time every candidate (tile_vertices, blocks_per_cu) on this batch and keep
 * the fastest; *best_ms (nullable) receives its run time. */
int pg_batch_autotune(pg_batch* bt, int estimator, void* stream, double* best_ms);
int pg_batch_destroy(pg_batch* bt);

/* ---- measurement ----------------------------------------------------------- */
typedef struct pg_kernel_time {
  char name[48];     /* launch site, e.g. "bf_build", "pairs_sum" */
  int64_t launches;  /* launches recorded since the last reset */
  double total_ms;   /* summed device time between HIP events recorded on the launch stream */
} pg_kernel_time;

/* Per-kernel device timing: while enabled, every kernel launch of the library
 * is bracketed by two HIP events on its stream. Process-wide. */
int pg_profile_enable(pg_ctx* ctx, int enable);
/* Record only the launch site `name` (host string, copied; NULL: every site).
 * Each recorded launch adds two events to its stream, which costs device time
 * between launches; selecting one site keeps that cost off the others. */
int pg_profile_select(pg_ctx* ctx, const char* name);
/* Wait for the recorded events and return up to `capacity` entries (host
 * array); *count receives the number of distinct launch sites. */
int pg_profile_read(pg_ctx* ctx, pg_kernel_time* out, int capacity, int* count);
int pg_profile_reset(pg_ctx* ctx);

/* Reference copy kernel: dst[i] = src[i] for `bytes` bytes (16-byte aligned
 * device buffers, bytes a multiple of 16). Used to calibrate HBM byte
 * counters and to measure the achievable copy bandwidth. */
int pg_copy(pg_ctx* ctx, void* dst, const void* src, size_t bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PROBGRAPH_H */
