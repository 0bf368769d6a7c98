/*
 * ProbGraph reference oracle: plain, slow, obviously correct CPU code.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load or call this file's library. The GPU
 * library never links, includes or calls it, and this file includes nothing
 * from the GPU library.
 *
 * Every loop follows the definition it cites, with no blocking or fusion. The
 * only parallelism is OpenMP over independent vertices or pairs (each
 * iteration writes its own output slot), so results do not depend on the
 * thread count.
 *
 * Graph: CSR with int32 offsets[n+1] and sorted, symmetric int32 adj[nnz]
 * (Section 2.1). Estimator formulas live in the Python half of the oracle
 * (FP64 numpy); this file produces the integer quantities they consume.
 *
 * Hashing (the paper uses MurmurHash3 with a time seed, Section 7; this
 * oracle follows the seeded multiply-add family chosen for the GPU library):
 *   SplitMix64 stream:  sm(key, i) = mix(key + (i+1) * 0x9E3779B97F4A7C15)
 *   constants of kind K: key = seed ^ tag(K);  a_i = sm(key, 2i) | 1,
 *                        c_i = sm(key, 2i+1)
 *   g_i(x) = a_i * x + c_i (mod 2^64), x the zero-extended 32-bit vertex ID
 *   Bloom-filter bit:    idx_i(x) = ((g_i(x) >> 32) * B) >> 32   (in [0, B))
 *                        word idx >> 6, bit idx & 63 (least significant first)
 *   MinHash key:         key_i(x) = mix(g_i(x)), a bijection of 64-bit words,
 *                        so two different vertices never tie.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_BOTTOM 0xFFFFFFFFu

/* Domain tags of the three sketch kinds. */
#define OR_TAG_BF 0x42462D48ull  /* "BF-H" */
#define OR_TAG_KH 0x4B482D48ull  /* "KH-H" */
#define OR_TAG_1H 0x31482D48ull  /* "1H-H" */

/* Threads an OpenMP loop of this library uses (reported with CPU timings). */
int or_threads(void) { return omp_get_max_threads(); }

/* Set the threads of later parallel loops (timing on one core, or all). */
void or_set_threads(int count) {
  if (count > 0) omp_set_num_threads(count);
}

/* ---------------------------------------------------------------- hashing */

static uint64_t or_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t or_splitmix64(uint64_t key, uint64_t i) {
  return or_mix(key + (i + 1) * 0x9E3779B97F4A7C15ull);
}

static uint64_t or_tag(int kind) {
  return kind == 1 ? OR_TAG_BF : kind == 2 ? OR_TAG_KH : OR_TAG_1H;
}

/* kind: 1 = Bloom filter, 2 = k-hash MinHash, 3 = 1-hash MinHash. */
void or_hash_consts(int kind, uint64_t seed, int count, uint64_t* a, uint64_t* c) {
  const uint64_t key = seed ^ or_tag(kind);
  for (int i = 0; i < count; ++i) {
    a[i] = or_splitmix64(key, 2 * (uint64_t)i) | 1ull;
    c[i] = or_splitmix64(key, 2 * (uint64_t)i + 1);
  }
}

uint32_t or_bf_index(uint64_t a, uint64_t c, uint32_t x, uint32_t B) {
  const uint64_t g = a * (uint64_t)x + c;
  return (uint32_t)(((g >> 32) * (uint64_t)B) >> 32);
}

uint64_t or_mh_key(uint64_t a, uint64_t c, uint32_t x) { return or_mix(a * (uint64_t)x + c); }

/* ------------------------------------------------------------ graph basics */

/* The m undirected edges, each once as (v, u) with v < u, in CSR order
 * (|E| = m, Section 2.1). eu/ev may be NULL to count only. */
int64_t or_upper_edges(int32_t n, const int32_t* off, const int32_t* adj, int32_t* eu, int32_t* ev) {
  int64_t m = 0;
  for (int32_t v = 0; v < n; ++v)
    for (int32_t p = off[v]; p < off[v + 1]; ++p)
      if (adj[p] > v) {
        if (eu) {
          eu[m] = v;
          ev[m] = adj[p];
        }
        ++m;
      }
  return m;
}

/* ------------------------------------------------------------ exact counts */

/* |N_u intersect N_v| by merging the two sorted neighbour lists (Fig. 1 and
 * the exact rows of Table "tab:queries-int"). */
static uint32_t or_merge_count(const int32_t* a, int32_t na, const int32_t* b, int32_t nb) {
  int32_t i = 0, j = 0;
  uint32_t cnt = 0;
  while (i < na && j < nb) {
    if (a[i] < b[j])
      ++i;
    else if (a[i] > b[j])
      ++j;
    else {
      ++cnt;
      ++i;
      ++j;
    }
  }
  return cnt;
}

void or_exact_pairs(int32_t n, const int32_t* off, const int32_t* adj, int64_t npairs, const int32_t* pu,
                    const int32_t* pv, uint32_t* out) {
  (void)n;
  int64_t e;
#pragma omp parallel for schedule(dynamic, 256)
  for (e = 0; e < npairs; ++e) {
    const int32_t u = pu[e], v = pv[e];
    out[e] = or_merge_count(adj + off[u], off[u + 1] - off[u], adj + off[v], off[v + 1] - off[v]);
  }
}

/* Node-iterator triangle count (Listing "lst:tc"): order R by (degree, ID)
 * ascending, N+_v = {u in N_v : R(v) < R(u)}, tc = sum over v, u in N+_v of
 * |N+_v intersect N+_u|. The N+ lists keep ID order, so merging applies. */
static int or_rank_less(const int32_t* off, int32_t v, int32_t u) {
  const int32_t dv = off[v + 1] - off[v], du = off[u + 1] - off[u];
  return dv < du || (dv == du && v < u);
}

uint64_t or_exact_tc_listing(int32_t n, const int32_t* off, const int32_t* adj) {
  int32_t* poff = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  int64_t total = 0;
  for (int32_t v = 0; v < n; ++v) {
    poff[v] = (int32_t)total;
    for (int32_t p = off[v]; p < off[v + 1]; ++p)
      if (or_rank_less(off, v, adj[p])) ++total;
  }
  poff[n] = (int32_t)total;
  int32_t* padj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
  for (int32_t v = 0; v < n; ++v) {
    int32_t q = poff[v];
    for (int32_t p = off[v]; p < off[v + 1]; ++p)
      if (or_rank_less(off, v, adj[p])) padj[q++] = adj[p];
  }
  uint64_t tc = 0;
  int32_t v;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : tc)
  for (v = 0; v < n; ++v)
    for (int32_t p = poff[v]; p < poff[v + 1]; ++p) {
      const int32_t u = padj[p];
      tc += or_merge_count(padj + poff[v], poff[v + 1] - poff[v], padj + poff[u], poff[u + 1] - poff[u]);
    }
  free(padj);
  free(poff);
  return tc;
}

/* ------------------------------------------------------------- 4-cliques */

static int or_rank_below(const int32_t* deg, int32_t v, int32_t u) {
  return deg[v] < deg[u] || (deg[v] == deg[u] && v < u);
}

/* Reformulated 4-clique count (Listing "lst:fcl"). With the degree order R of
 * the triangle count and the lists N+_v (ID order) given as poff/padj: for
 * every u and v in N+_u, C3 = N+_u intersect N+_v; for every w in C3 add
 * |N+_w intersect C3|. A 4-clique is counted once, at its three lowest-ranked
 * vertices. deg holds the full degrees (the order R).
 *
 * With words != NULL (Bloom filters of the N+ sets: B bits, b hash functions
 * of seed) |N+_w intersect C3| is replaced by the number of x in C3 ranked
 * above w whose b bits are all set in the filter of N+_w: a membership query
 * per element (Section 2.4), answered with false positives only. */
uint64_t or_four_cliques(int32_t n, const int32_t* poff, const int32_t* padj, const int32_t* deg,
                         const uint64_t* words, uint32_t B, uint32_t b, uint64_t seed) {
  int32_t maxd = 0;
  for (int32_t v = 0; v < n; ++v)
    if (poff[v + 1] - poff[v] > maxd) maxd = poff[v + 1] - poff[v];
  const uint32_t W = B / 64;
  uint64_t a[64], c[64];
  if (words) or_hash_consts(1, seed, (int)b, a, c);
  uint64_t total = 0;
#pragma omp parallel reduction(+ : total)
  {
    int32_t* c3 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(maxd > 0 ? maxd : 1));
    int32_t u;
#pragma omp for schedule(dynamic, 64)
    for (u = 0; u < n; ++u) {
      for (int32_t p = poff[u]; p < poff[u + 1]; ++p) {
        const int32_t v = padj[p];
        /* C3 by merging N+_u and N+_v (both in ID order) */
        int32_t i = poff[u], j = poff[v], s = 0;
        while (i < poff[u + 1] && j < poff[v + 1]) {
          if (padj[i] < padj[j])
            ++i;
          else if (padj[i] > padj[j])
            ++j;
          else {
            c3[s++] = padj[i];
            ++i;
            ++j;
          }
        }
        for (int32_t t = 0; t < s; ++t) {
          const int32_t w = c3[t];
          if (!words) {
            total += or_merge_count(padj + poff[w], poff[w + 1] - poff[w], c3, s);
            continue;
          }
          const uint64_t* bw = words + (size_t)w * W;
          for (int32_t q = 0; q < s; ++q) {
            const int32_t x = c3[q];
            if (!or_rank_below(deg, w, x)) continue;
            int member = 1;
            for (uint32_t h = 0; h < b && member; ++h) {
              const uint32_t idx = or_bf_index(a[h], c[h], (uint32_t)x, B);
              member = (int)((bw[idx >> 6] >> (idx & 63)) & 1ull);
            }
            total += (uint64_t)member;
          }
        }
      }
    }
    free(c3);
  }
  return total;
}

/* 4-cliques with |N+_w intersect C3| estimated from two Bloom filters (the
 * sketch-intersection form of Listing "lst:fcl", whose work bound counts
 * B/W word operations per w): the filter of N+_w (words, B bits, b hash
 * functions of seed) and, for each oriented edge, the filter of C3 built
 * with the same functions. c is the number of ones of their AND and c_or of
 * their OR. The AND, limit and existing-filter estimators are functions of c
 * alone and the OR estimator of c_or and the sizes |N+_w| + |C3|, so the
 * routine returns how often each value occurs over all (edge, w in C3):
 * hist_and[c] and hist_or[c_or] (B + 1 entries each, overwritten), and the
 * sum of |N+_w| + |C3| in *sizes. Every w in C3 takes part (no rank test):
 * the filter of N+_w holds only vertices ranked above w anyway. */
void or_four_cliques_filters(int32_t n, const int32_t* poff, const int32_t* padj, const uint64_t* words, uint32_t B,
                             uint32_t b, uint64_t seed, uint64_t* hist_and, uint64_t* hist_or, uint64_t* sizes) {
  int32_t maxd = 0;
  for (int32_t v = 0; v < n; ++v)
    if (poff[v + 1] - poff[v] > maxd) maxd = poff[v + 1] - poff[v];
  const uint32_t W = B / 64;
  uint64_t a[64], c[64];
  or_hash_consts(1, seed, (int)b, a, c);
  for (uint32_t t = 0; t <= B; ++t) hist_and[t] = hist_or[t] = 0;
  uint64_t size_sum = 0;
#pragma omp parallel reduction(+ : size_sum)
  {
    int32_t* c3 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(maxd > 0 ? maxd : 1));
    uint64_t* f = (uint64_t*)malloc(sizeof(uint64_t) * W);
    uint64_t* ha = (uint64_t*)calloc((size_t)B + 1, sizeof(uint64_t));
    uint64_t* ho = (uint64_t*)calloc((size_t)B + 1, sizeof(uint64_t));
    int32_t u;
#pragma omp for schedule(dynamic, 64)
    for (u = 0; u < n; ++u) {
      for (int32_t p = poff[u]; p < poff[u + 1]; ++p) {
        const int32_t v = padj[p];
        int32_t i = poff[u], j = poff[v], s = 0;
        while (i < poff[u + 1] && j < poff[v + 1]) {
          if (padj[i] < padj[j])
            ++i;
          else if (padj[i] > padj[j])
            ++j;
          else {
            c3[s++] = padj[i];
            ++i;
            ++j;
          }
        }
        if (s == 0) continue;
        for (uint32_t q = 0; q < W; ++q) f[q] = 0;
        for (int32_t t = 0; t < s; ++t)
          for (uint32_t h = 0; h < b; ++h) {
            const uint32_t idx = or_bf_index(a[h], c[h], (uint32_t)c3[t], B);
            f[idx >> 6] |= 1ull << (idx & 63);
          }
        for (int32_t t = 0; t < s; ++t) {
          const int32_t w = c3[t];
          const uint64_t* bw = words + (size_t)w * W;
          uint32_t ones_and = 0, ones_or = 0;
          for (uint32_t q = 0; q < W; ++q) {
            ones_and += (uint32_t)__builtin_popcountll(bw[q] & f[q]);
            ones_or += (uint32_t)__builtin_popcountll(bw[q] | f[q]);
          }
          ++ha[ones_and];
          ++ho[ones_or];
          size_sum += (uint64_t)(poff[w + 1] - poff[w]) + (uint64_t)s;
        }
      }
    }
#pragma omp critical
    for (uint32_t t = 0; t <= B; ++t) {
      hist_and[t] += ha[t];
      hist_or[t] += ho[t];
    }
    free(ho);
    free(ha);
    free(f);
    free(c3);
  }
  *sizes = size_sum;
}

/* ----------------------------------------------------------- Bloom filters */

/* B_v: B bits (W = B/64 words), for each x in N_v and each of the b hash
 * functions set bit idx_i(x) (Section 2.4, "Bloom filters"). pc[v] is the
 * number of ones, B_{v,1}. */
void or_bf_build(int32_t n, const int32_t* off, const int32_t* adj, uint32_t B, uint32_t b, uint64_t seed,
                 uint64_t* words, uint32_t* pc) {
  const uint32_t W = B / 64;
  uint64_t* a = (uint64_t*)malloc(sizeof(uint64_t) * b);
  uint64_t* c = (uint64_t*)malloc(sizeof(uint64_t) * b);
  or_hash_consts(1, seed, (int)b, a, c);
  int32_t v;
#pragma omp parallel for schedule(dynamic, 256)
  for (v = 0; v < n; ++v) {
    uint64_t* bv = words + (size_t)v * W;
    for (uint32_t w = 0; w < W; ++w) bv[w] = 0;
    for (int32_t p = off[v]; p < off[v + 1]; ++p)
      for (uint32_t i = 0; i < b; ++i) {
        const uint32_t idx = or_bf_index(a[i], c[i], (uint32_t)adj[p], B);
        bv[idx >> 6] |= 1ull << (idx & 63);
      }
    uint32_t ones = 0;
    for (uint32_t w = 0; w < W; ++w) ones += (uint32_t)__builtin_popcountll(bv[w]);
    pc[v] = ones;
  }
  free(a);
  free(c);
}

/* The Bloom filter of an arbitrary set (same hash functions), for tests. */
void or_bf_of_set(int32_t len, const int32_t* xs, uint32_t B, uint32_t b, uint64_t seed, uint64_t* words) {
  const uint32_t W = B / 64;
  uint64_t a[64], c[64];
  or_hash_consts(1, seed, (int)b, a, c);
  for (uint32_t w = 0; w < W; ++w) words[w] = 0;
  for (int32_t t = 0; t < len; ++t)
    for (uint32_t i = 0; i < b; ++i) {
      const uint32_t idx = or_bf_index(a[i], c[i], (uint32_t)xs[t], B);
      words[idx >> 6] |= 1ull << (idx & 63);
    }
}

/* c = ones of (B_u AND B_v), the approximation of B_{X cap Y} used by the
 * AND estimator (Section 4.2); c_or = ones of (B_u OR B_v) (Section 8.1).
 * Either output may be NULL. */
void or_bf_counts(uint32_t W, const uint64_t* words, int64_t npairs, const int32_t* pu, const int32_t* pv,
                  uint32_t* c_and, uint32_t* c_or) {
  int64_t e;
#pragma omp parallel for schedule(static)
  for (e = 0; e < npairs; ++e) {
    const uint64_t* bu = words + (size_t)pu[e] * W;
    const uint64_t* bv = words + (size_t)pv[e] * W;
    uint32_t x = 0, y = 0;
    for (uint32_t w = 0; w < W; ++w) {
      x += (uint32_t)__builtin_popcountll(bu[w] & bv[w]);
      y += (uint32_t)__builtin_popcountll(bu[w] | bv[w]);
    }
    if (c_and) c_and[e] = x;
    if (c_or) c_or[e] = y;
  }
}

/* ------------------------------------------------------ MinHash, k-hash */

/* For each of the k hash functions separately, the element of N_v with the
 * smallest hash (Section 2.4, "MinHash (k-Hash variant)"); duplicates across
 * positions are allowed. Empty N_v gives the bottom marker in every slot. */
void or_kh_build(int32_t n, const int32_t* off, const int32_t* adj, uint32_t k, uint64_t seed, uint32_t* sig) {
  uint64_t* a = (uint64_t*)malloc(sizeof(uint64_t) * k);
  uint64_t* c = (uint64_t*)malloc(sizeof(uint64_t) * k);
  or_hash_consts(2, seed, (int)k, a, c);
  int32_t v;
#pragma omp parallel for schedule(dynamic, 256)
  for (v = 0; v < n; ++v)
    for (uint32_t i = 0; i < k; ++i) {
      uint32_t best = OR_BOTTOM;
      uint64_t best_key = 0;
      for (int32_t p = off[v]; p < off[v + 1]; ++p) {
        const uint32_t x = (uint32_t)adj[p];
        const uint64_t key = or_mh_key(a[i], c[i], x);
        if (best == OR_BOTTOM || key < best_key || (key == best_key && x < best)) {
          best = x;
          best_key = key;
        }
      }
      sig[(size_t)v * k + i] = best;
    }
  free(a);
  free(c);
}

/* s = number of positions i with M_u[i] == M_v[i] (positional comparison,
 * which is the Bin(k, J) count of Section 4.3); the bottom marker never
 * matches. */
void or_kh_counts(uint32_t k, const uint32_t* sig, int64_t npairs, const int32_t* pu, const int32_t* pv,
                  uint32_t* s) {
  int64_t e;
#pragma omp parallel for schedule(static)
  for (e = 0; e < npairs; ++e) {
    const uint32_t* mu = sig + (size_t)pu[e] * k;
    const uint32_t* mv = sig + (size_t)pv[e] * k;
    uint32_t cnt = 0;
    for (uint32_t i = 0; i < k; ++i)
      if (mu[i] == mv[i] && mu[i] != OR_BOTTOM) ++cnt;
    s[e] = cnt;
  }
}

/* ------------------------------------------------------ MinHash, 1-hash */

typedef struct {
  uint64_t key;
  uint32_t x;
} or_keyed;

static int or_keyed_cmp(const void* pa, const void* pb) {
  const or_keyed* a = (const or_keyed*)pa;
  const or_keyed* b = (const or_keyed*)pb;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  return a->x < b->x ? -1 : (a->x > b->x ? 1 : 0);
}

/* The min(k, d_v) elements of N_v with the smallest values of the single hash
 * (Section 2.4, "MinHash (1-Hash variant)"), stored in ascending hash order,
 * padded with the bottom marker. */
void or_1h_build(int32_t n, const int32_t* off, const int32_t* adj, uint32_t k, uint64_t seed, uint32_t* sig) {
  uint64_t a, c;
  or_hash_consts(3, seed, 1, &a, &c);
  int32_t v;
#pragma omp parallel for schedule(dynamic, 256)
  for (v = 0; v < n; ++v) {
    const int32_t d = off[v + 1] - off[v];
    or_keyed* tmp = (or_keyed*)malloc(sizeof(or_keyed) * (size_t)(d > 0 ? d : 1));
    for (int32_t t = 0; t < d; ++t) {
      tmp[t].x = (uint32_t)adj[off[v] + t];
      tmp[t].key = or_mh_key(a, c, tmp[t].x);
    }
    qsort(tmp, (size_t)d, sizeof(or_keyed), or_keyed_cmp);
    for (uint32_t i = 0; i < k; ++i) sig[(size_t)v * k + i] = (int32_t)i < d ? tmp[i].x : OR_BOTTOM;
    free(tmp);
  }
}

/* Per pair, with M_u and M_v the two 1-hash sets:
 *   s_lit  = |M_u intersect M_v|                      (literal reading)
 *   kprime = min(k, |M_u union M_v|)
 *   s_uni  = |U intersect M_u intersect M_v|, U the kprime elements of
 *            M_u union M_v with the smallest hash   (bottom-k of the union)
 * The second reading is the one whose count is hypergeometric with
 * population |X union Y| (Section 4.4). Walks both lists in hash order. */
void or_1h_counts(uint32_t k, uint64_t seed, const uint32_t* sig, int64_t npairs, const int32_t* pu,
                  const int32_t* pv, uint32_t* s_uni, uint32_t* kprime, uint32_t* s_lit) {
  uint64_t a, c;
  or_hash_consts(3, seed, 1, &a, &c);
  int64_t e;
#pragma omp parallel for schedule(static)
  for (e = 0; e < npairs; ++e) {
    const uint32_t* mu = sig + (size_t)pu[e] * k;
    const uint32_t* mv = sig + (size_t)pv[e] * k;
    uint32_t nu = 0, nv = 0;
    while (nu < k && mu[nu] != OR_BOTTOM) ++nu;
    while (nv < k && mv[nv] != OR_BOTTOM) ++nv;
    /* literal intersection size */
    uint32_t common = 0;
    for (uint32_t i = 0; i < nu; ++i)
      for (uint32_t j = 0; j < nv; ++j)
        if (mu[i] == mv[j]) ++common;
    const uint32_t uni = nu + nv - common;
    const uint32_t kp = uni < k ? uni : k;
    /* the kp smallest of the union, in hash order */
    uint32_t i = 0, j = 0, taken = 0, su = 0;
    while (taken < kp) {
      const uint64_t ku = i < nu ? or_mh_key(a, c, mu[i]) : UINT64_MAX;
      const uint64_t kv = j < nv ? or_mh_key(a, c, mv[j]) : UINT64_MAX;
      if (i < nu && j < nv && mu[i] == mv[j]) {
        ++su;
        ++i;
        ++j;
      } else if (j >= nv || (i < nu && ku < kv)) {
        ++i;
      } else {
        ++j;
      }
      ++taken;
    }
    if (s_uni) s_uni[e] = su;
    if (kprime) kprime[e] = kp;
    if (s_lit) s_lit[e] = common;
  }
}
