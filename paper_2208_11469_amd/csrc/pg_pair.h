// Per-pair intersection estimates (Sections 4.2-4.4), shared by the batch
// kernels of the estimate path and of the serving engine.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pg_device.h"
#include "probgraph.h"

struct pg_sketches;

namespace pg {

struct SkView {
  int kind;
  int est;
  uint32_t size;  // B or k
  uint32_t b;
  uint32_t W;
  int32_t n;
  const uint64_t* words;
  const uint32_t* pc;
  const uint32_t* sig;
  const double* table;
  const int32_t* deg;
  uint64_t a1, c1;  // 1-hash constants
};

// ---- integer counts ----------------------------------------------------------

template <int WT>
__device__ __forceinline__ uint32_t bf_and_count(const uint64_t* __restrict__ ru, const uint64_t* __restrict__ rv,
                                                 uint32_t W) {
  uint32_t c = 0;
  if constexpr (WT > 0 && (WT % 2) == 0) {
    // rows of an even word count start on 16-byte boundaries
    const ulonglong2* u2 = reinterpret_cast<const ulonglong2*>(ru);
    const ulonglong2* v2 = reinterpret_cast<const ulonglong2*>(rv);
#pragma unroll
    for (int j = 0; j < WT / 2; ++j) {
      const ulonglong2 x = u2[j], y = v2[j];
      c += (uint32_t)__popcll(x.x & y.x) + (uint32_t)__popcll(x.y & y.y);
    }
  } else if constexpr (WT > 0) {
#pragma unroll
    for (int j = 0; j < WT; ++j) c += (uint32_t)__popcll(ru[j] & rv[j]);
  } else {
    for (uint32_t j = 0; j < W; ++j) c += (uint32_t)__popcll(ru[j] & rv[j]);
  }
  return c;
}

__device__ __forceinline__ uint32_t kh_matches(const uint32_t* __restrict__ mu, const uint32_t* __restrict__ mv,
                                               uint32_t k) {
  uint32_t s = 0;
  if ((k & 3u) == 0) {
    const uint4* u4 = reinterpret_cast<const uint4*>(mu);
    const uint4* v4 = reinterpret_cast<const uint4*>(mv);
    for (uint32_t j = 0; j < k / 4; ++j) {
      const uint4 x = u4[j], y = v4[j];
      s += (x.x == y.x && x.x != kBottom) + (x.y == y.y && x.y != kBottom) + (x.z == y.z && x.z != kBottom) +
           (x.w == y.w && x.w != kBottom);
    }
  } else {
    for (uint32_t j = 0; j < k; ++j) s += (mu[j] == mv[j] && mu[j] != kBottom);
  }
  return s;
}

// Walk of two 1-hash rows (each ascending in key) in key order.
//   common      = |M_u cap M_v|
//   kprime      = min(k, |M_u cup M_v|)
//   s_union     = commons among the kprime smallest of the union
//   kth_key     = key of the k-th smallest element of the union (~0 if fewer)
__device__ __forceinline__ void oh_counts(const uint32_t* __restrict__ mu, const uint32_t* __restrict__ mv, uint32_t k,
                                          uint32_t nu, uint32_t nv, uint64_t a, uint64_t c, uint32_t& s_union,
                                          uint32_t& kprime, uint32_t& common, uint64_t& kth_key) {
  uint32_t i = 0, j = 0, rank = 0, com = 0, com_k = 0;
  uint64_t ku = nu ? mh_key(a, c, mu[0]) : ~0ull;
  uint64_t kv = nv ? mh_key(a, c, mv[0]) : ~0ull;
  uint64_t kth = ~0ull;
  while (i < nu || j < nv) {
    uint64_t cur;
    if (i < nu && j < nv && mu[i] == mv[j]) {
      cur = ku;
      com_k += rank < k ? 1u : 0u;
      ++com;
      ++i;
      ++j;
      ku = i < nu ? mh_key(a, c, mu[i]) : ~0ull;
      kv = j < nv ? mh_key(a, c, mv[j]) : ~0ull;
    } else if (j >= nv || (i < nu && ku < kv)) {
      cur = ku;
      ++i;
      ku = i < nu ? mh_key(a, c, mu[i]) : ~0ull;
    } else {
      cur = kv;
      ++j;
      kv = j < nv ? mh_key(a, c, mv[j]) : ~0ull;
    }
    if (rank + 1 == k) kth = cur;
    ++rank;
  }
  const uint32_t uni = nu + nv - com;
  kprime = uni < k ? uni : k;
  s_union = uni >= k ? com_k : com;
  common = com;
  kth_key = kth;
}

// KMV hash in (0, 1]: the top 53 bits of a MinHash key, plus one, times 2^-53.
__device__ __forceinline__ double kmv_hash(uint64_t key) {
  return (double)((key >> 11) + 1ull) * 0x1.0p-53;
}

// KMV estimate of |X cap Y| (Section "Beyond Bloom Filter and MinHash",
// Eqs. "est_inter_set_kmv_exactsets" and "est_inter_set_kmv"): nx, ny values
// in the rows (min(k, d)), uni = |M_X u M_Y|, kth_key the k-th smallest union
// key, max_x / max_y the largest key of each row.
__device__ __forceinline__ double kmv_estimate(bool exact_sizes, uint32_t k, int32_t dx, int32_t dy, uint32_t nx,
                                               uint32_t ny, uint32_t uni, uint64_t kth_key, uint64_t max_x,
                                               uint64_t max_y) {
  if (dx == 0 || dy == 0) return 0.0;
  const double km1 = (double)k - 1.0;
  const double u_hat = (nx < k && ny < k) ? (double)uni : km1 / kmv_hash(kth_key);
  if (exact_sizes) return ((double)dx + (double)dy) - u_hat;
  const double sx = nx < k ? (double)nx : km1 / kmv_hash(max_x);
  const double sy = ny < k ? (double)ny : km1 / kmv_hash(max_y);
  return (sx + sy) - u_hat;
}

// J^ = s / kk, I^ = J^ / (1 + J^) (|X| + |Y|)  (Eq. "est_int_mh", Section 4.4)
__device__ __forceinline__ double minhash_estimate(uint32_t s, uint32_t kk, int32_t du, int32_t dv) {
  const double j = kk > 0 ? (double)s / (double)kk : 0.0;
  return j / (1.0 + j) * ((double)du + (double)dv);
}

template <int KIND, int WT>
__device__ __forceinline__ double eval_pair(const SkView& s, int32_t u, int32_t v, uint32_t& raw) {
  if ((uint32_t)u >= (uint32_t)s.n || (uint32_t)v >= (uint32_t)s.n) {
    raw = 0xFFFFFFFFu;
    return __longlong_as_double(0x7FF8000000000000ll);  // NaN for an out-of-range pair
  }
  if constexpr (KIND == PG_BF) {
    const uint32_t W = WT > 0 ? (uint32_t)WT : s.W;
    const uint32_t c = bf_and_count<WT>(s.words + bf_row_offset(u, W), s.words + bf_row_offset(v, W), W);
    if (s.est == PG_EST_BF_OR) {
      const uint32_t cor = s.pc[u] + s.pc[v] - c;  // ones of the OR
      raw = cor;
      return ((double)s.deg[u] + (double)s.deg[v]) + s.table[cor];
    }
    raw = c;
    return s.table[c];
  } else if constexpr (KIND == PG_MH_KHASH) {
    const uint32_t m = kh_matches(s.sig + (size_t)u * s.size, s.sig + (size_t)v * s.size, s.size);
    raw = m;
    return minhash_estimate(m, s.size, s.deg[u], s.deg[v]);
  } else {
    const int32_t du = s.deg[u], dv = s.deg[v];
    const uint32_t nu = (uint32_t)du < s.size ? (uint32_t)du : s.size;
    const uint32_t nv = (uint32_t)dv < s.size ? (uint32_t)dv : s.size;
    uint32_t su, kp, com;
    uint64_t kth;
    const uint32_t* mu = s.sig + (size_t)u * s.size;
    const uint32_t* mv = s.sig + (size_t)v * s.size;
    oh_counts(mu, mv, s.size, nu, nv, s.a1, s.c1, su, kp, com, kth);
    if (s.est == PG_EST_KMV || s.est == PG_EST_KMV_SKETCH_SIZES) {
      raw = kp;
      const bool exact_sizes = s.est == PG_EST_KMV;
      const uint64_t max_u = (!exact_sizes && nu) ? mh_key(s.a1, s.c1, mu[nu - 1]) : 0ull;
      const uint64_t max_v = (!exact_sizes && nv) ? mh_key(s.a1, s.c1, mv[nv - 1]) : 0ull;
      return kmv_estimate(exact_sizes, s.size, du, dv, nu, nv, nu + nv - com, kth, max_u, max_v);
    }
    if (s.est == PG_EST_MH_1HASH_LITERAL) {
      raw = com;
      return minhash_estimate(com, s.size, du, dv);
    }
    raw = su;
    return minhash_estimate(su, kp, du, dv);
  }
}

// Similarity of N_u and N_v from an intersection value I (Listing "lst:sim"):
// common neighbours I itself; for the others I_c = clamp(I, 0, min(d_u, d_v)),
// Jaccard I_c / (d_u + d_v - I_c) (0 on an empty union), overlap
// I_c / min(d_u, d_v) (0 when the smaller set is empty), total neighbours
// d_u + d_v - I_c.
__device__ __forceinline__ double similarity_of(int measure, double est, int32_t du, int32_t dv) {
  if (measure == PG_SIM_COMMON) return est;
  const double hi = (double)(du < dv ? du : dv);
  const double ic = est < 0.0 ? 0.0 : (est > hi ? hi : est);
  const double sum = (double)du + (double)dv;
  if (measure == PG_SIM_JACCARD) {
    const double den = sum - ic;
    return den > 0.0 ? ic / den : 0.0;
  }
  if (measure == PG_SIM_OVERLAP) return hi > 0.0 ? ic / hi : 0.0;
  return sum - ic;  // PG_SIM_TOTAL
}

__device__ __forceinline__ double jaccard_of(double est, int32_t du, int32_t dv) {
  return similarity_of(PG_SIM_JACCARD, est, du, dv);
}


// Kind chosen at run time (mixed batches); Bloom filters use the general word loop.
__device__ __forceinline__ double eval_pair_any(const SkView& s, int32_t u, int32_t v, uint32_t& raw) {
  if (s.kind == PG_BF) return eval_pair<PG_BF, 0>(s, u, v, raw);
  if (s.kind == PG_MH_KHASH) return eval_pair<PG_MH_KHASH, 0>(s, u, v, raw);
  return eval_pair<PG_MH_1HASH, 0>(s, u, v, raw);
}

// Host side (pg_estimate.hip): the view of a sketch set for an estimator, and
// the check that the estimator applies to the sketch kind.
SkView make_view(const pg_sketches* sk, int est);
int check_estimator(const pg_sketches* sk, int est);

}  // namespace pg
