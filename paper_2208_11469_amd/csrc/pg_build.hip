// Sketch construction (Section 2.4; work and depth in Table "tab:constr").
//
// Bloom filter: every element x of N_v sets bit idx_i(x) for each of b hash
// functions. k-hash: for each hash function i, the element of N_v with the
// smallest key_i. 1-hash: the min(k, d_v) elements of N_v with the smallest
// key, in ascending key order.
//
// Vertices are processed by groups of G lanes, G growing with the degree.
// Filters: the lanes of a group set bits in one shared LDS bitmap with atomic
// OR. k-hash: every lane keeps private minima over a strided slice of N_v in
// registers, combined by a fixed butterfly (lexicographic (key, ID) minimum).
// Both combinations are order-independent, so the result does not depend on
// scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "pg_device.h"
#include "pg_internal.h"

namespace pg {
namespace {

constexpr int kBlock = 256;

// ---------------------------------------------------------------- Bloom filter

// ---- Bloom filter over a vertex work plan (W <= 16 words) -------------------
//
// One launch, three tiers (heavy chunks first): heavy vertices are split into
// chunks of kHeavyChunk arcs, one block each; medium vertices get a wave;
// light vertices (at most kLightMax neighbours) get kLightGroup lanes each.
//
// Bit scatter: the lanes serving one vertex share one W-word bitmap in LDS and
// set the bit of each hashed neighbour with an LDS atomic OR (one LDS
// instruction per hash, no read-modify-write round trip). OR is commutative
// and idempotent, so the bitmap does not depend on the order in which lanes
// land. Each lane issues U neighbour loads before hashing any of them. The
// group then writes its bitmap out as the row, W lanes one word each. Waves
// and blocks (medium and heavy tiers) keep kBfCopies bitmaps, lane l using
// copy l mod kBfCopies, so that fewer lanes of one instruction collide on the
// same word; the copies are OR-ed when the row is written.
constexpr int kBfCopies = 8;

template <int U, int G>
__device__ __forceinline__ void bf_scatter(const int32_t* __restrict__ adj, int64_t beg, int64_t end, int lane,
                                           uint32_t B, uint32_t b, const uint64_t* __restrict__ ha,
                                           const uint64_t* __restrict__ hc, uint64_t* __restrict__ bits) {
  for (int64_t p0 = beg + lane; p0 < end; p0 += (int64_t)G * U) {
    uint32_t x[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int64_t p = p0 + (int64_t)j * G;
      x[j] = p < end ? (uint32_t)adj[p] : 0u;
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      if (p0 + (int64_t)j * G < end) {
        for (uint32_t i = 0; i < b; ++i) {
          const uint32_t idx = bf_index(ha[i], hc[i], x[j], B);
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

template <int W>
__global__ __launch_bounds__(kBlock) void k_bf_build_plan(PlanView P, const int32_t* __restrict__ off,
                                                          const int32_t* __restrict__ adj, uint32_t B, uint32_t b,
                                                          const uint64_t* __restrict__ ha,
                                                          const uint64_t* __restrict__ hc, uint64_t* __restrict__ words,
                                                          uint32_t* __restrict__ pc, uint64_t* __restrict__ part) {
  constexpr int kLightWords = (kBlock / kLightGroup) * W;       // one bitmap per light group
  constexpr int kWaveWords = (kBlock / kWave) * kBfCopies * W;  // kBfCopies bitmaps per wave (or per heavy block)
  __shared__ uint64_t lds[kLightWords > kWaveWords ? kLightWords : kWaveWords];
  const int64_t blk = blockIdx.x;
  const int tid = threadIdx.x;

  if (blk < P.n_chunks) {  // ---- heavy chunk: the whole block; partial row to `part`
    for (int i = tid; i < kBfCopies * W; i += kBlock) lds[i] = 0;
    __syncthreads();
    bf_scatter<8, kBlock>(adj, P.chunk_begin[blk], P.chunk_end[blk], tid, B, b, ha, hc,
                          lds + (tid % kBfCopies) * W);
    __syncthreads();
    if (tid < W) {
      uint64_t w = 0;
#pragma unroll
      for (int c = 0; c < kBfCopies; ++c) w |= lds[c * W + tid];
      part[blk * W + tid] = w;
    }
    return;
  }
  const int64_t mb = blk - P.n_chunks;
  if (mb < P.n_medium_blocks) {  // ---- medium: one wave per vertex
    const int wv = tid / kWave;
    const int lane = lane_id();
    uint64_t* bits = lds + wv * kBfCopies * W;
    const int64_t idx = mb * (kBlock / kWave) + wv;
    const bool active = idx < P.n_medium;
    const int32_t v = active ? P.medium[idx] : 0;
    for (int i = lane; i < kBfCopies * W; i += kWave) bits[i] = 0;
    wave_sync();
    if (active) bf_scatter<8, kWave>(adj, off[v], off[v + 1], lane, B, b, ha, hc, bits + (lane % kBfCopies) * W);
    wave_sync();
    uint32_t ones = 0;
    if (active && lane < W) {
      uint64_t w = 0;
#pragma unroll
      for (int c = 0; c < kBfCopies; ++c) w |= bits[c * W + lane];
      words[bf_row_offset(v, W) + lane] = w;
      ones = (uint32_t)__popcll(w);
    }
    ones = group_sum_u32<kWave>(ones);
    if (active && lane == 0) pc[v] = ones;
    return;
  }
  // ---- light: kLightGroup lanes per vertex of the light list (sorted by
  // degree, so the groups of a wave walk about equally many arcs)
  const int64_t idx = ((mb - P.n_medium_blocks) * kBlock + tid) / kLightGroup;
  const int lane = tid % kLightGroup;
  uint64_t* bits = lds + (tid / kLightGroup) * W;
  const bool active = idx < P.n_light;
  const int32_t v = active ? P.light[idx] : 0;
  const int64_t beg = active ? off[v] : 0, end = active ? off[v + 1] : 0;
  for (int k = lane; k < W; k += kLightGroup) bits[k] = 0;
  wave_sync();
  if (active) bf_scatter<kLightUnroll, kLightGroup>(adj, beg, end, lane, B, b, ha, hc, bits);
  wave_sync();
  uint32_t ones = 0;
  if (active) {
    uint64_t* row = words + bf_row_offset(v, W);
    for (int k = lane; k < W; k += kLightGroup) {
      const uint64_t w = bits[k];
      row[k] = w;
      ones += (uint32_t)__popcll(w);
    }
  }
  ones = group_sum_u32<kLightGroup>(ones);
  if (active && lane == 0) pc[v] = ones;
}

// Heavy vertices: OR of the chunk partials; one wave per vertex. Lane l reads
// word l mod W of every (64 / W)-th chunk starting at chunk l / W, so the
// wave reads 64 / W partial rows side by side; the lanes holding the same
// word then meet in LDS. OR is order-independent.
template <int W>
__global__ __launch_bounds__(kBlock) void k_bf_combine(PlanView P, const uint64_t* __restrict__ part, int64_t n_heavy,
                                                       uint64_t* __restrict__ words, uint32_t* __restrict__ pc) {
  __shared__ uint64_t lds[kBlock];
  const int64_t h = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / kWave;  // the same in every lane of a wave
  if (h >= n_heavy) return;
  const int lane = lane_id();
  constexpr int R = kWave / W;  // partial rows in flight
  const int word = lane % W, row = lane / W;
  const int32_t c0 = P.heavy_first[h], c1 = P.heavy_first[h + 1];
  const int32_t v = P.chunk_vertex[c0];
  uint64_t acc = 0;
  if (row < R)
    for (int32_t c = c0 + row; c < c1; c += R) acc |= part[(int64_t)c * W + word];
  uint64_t* mine = lds + (threadIdx.x / kWave) * kWave;
  mine[lane] = acc;
  wave_sync();
  uint64_t w = 0;
  if (lane < W) {
#pragma unroll
    for (int r = 0; r < R; ++r) w |= mine[r * W + lane];
    words[bf_row_offset(v, W) + lane] = w;
  }
  const uint32_t ones = group_sum_u32<kWave>((uint32_t)__popcll(w));
  if (lane == 0) pc[v] = ones;
}

// Filters wider than 16 words: one wave per vertex, lane w owns word w
// (W <= 64); every lane evaluates all hashes and keeps the bits of its word.
__global__ __launch_bounds__(kBlock) void k_bf_build_wide(const int32_t* __restrict__ off,
                                                          const int32_t* __restrict__ adj, int32_t n, uint32_t B,
                                                          uint32_t W, uint32_t b, const uint64_t* __restrict__ ha,
                                                          const uint64_t* __restrict__ hc, uint64_t* __restrict__ words,
                                                          uint32_t* __restrict__ pc) {
  const int64_t v = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / kWave;
  const int lane = lane_id();
  if (v >= n) return;
  uint64_t mine = 0;
  for (int64_t p = off[v]; p < off[v + 1]; ++p) {
    const uint32_t x = (uint32_t)adj[p];
    for (uint32_t i = 0; i < b; ++i) {
      const uint32_t idx = bf_index(ha[i], hc[i], x, B);
      if ((idx >> 6) == (uint32_t)lane) mine |= 1ull << (idx & 63u);
    }
  }
  if ((uint32_t)lane < W) words[bf_row_offset(v, W) + lane] = mine;
  const uint32_t ones = group_sum_u32<kWave>((uint32_t)__popcll(mine));
  if (lane == 0) pc[v] = ones;
}

// ---------------------------------------------------------------- k-hash

constexpr int kKhBatch = 8;  // hash functions kept in registers at a time (8: 2.71 ms, 4: 2.78, 16: 3.05, 32: 3.77 for k = 32 on R-MAT s20)

template <int G>
__device__ __forceinline__ void min_pair_group(uint64_t& key, uint32_t& id) {
#pragma unroll
  for (int s = G / 2; s >= 1; s >>= 1) {
    const uint64_t ok = __shfl_xor(key, s, G);
    const uint32_t oi = __shfl_xor(id, s, G);
    if (ok < key || (ok == key && oi < id)) {
      key = ok;
      id = oi;
    }
  }
}

// Vertices of one degree bin, G lanes each; vertices with more than max_deg
// arcs are left to the chunked kernels below.
template <int G>
__global__ __launch_bounds__(kBlock) void k_kh_build(const int32_t* __restrict__ off, const int32_t* __restrict__ adj,
                                                     const int32_t* __restrict__ verts, int64_t nverts, uint32_t k,
                                                     const uint64_t* __restrict__ ha, const uint64_t* __restrict__ hc,
                                                     uint32_t* __restrict__ sig, int64_t max_deg) {
  __shared__ uint64_t lkey[(G > kWave) ? (kBlock / kWave) * kKhBatch : 1];
  __shared__ uint32_t lid[(G > kWave) ? (kBlock / kWave) * kKhBatch : 1];
  const int64_t grp = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x % G;
  bool active = grp < nverts;
  const int32_t v = active ? verts[grp] : 0;
  const int64_t beg = active ? off[v] : 0;
  int64_t end = active ? off[v + 1] : 0;
  if (end - beg > max_deg) {  // chunked instead (the whole group skips it)
    active = false;
    end = beg;
  }
  for (uint32_t i0 = 0; i0 < k; i0 += kKhBatch) {
    uint64_t best[kKhBatch];
    uint32_t bid[kKhBatch];
#pragma unroll
    for (int j = 0; j < kKhBatch; ++j) {
      best[j] = ~0ull;
      bid[j] = kBottom;
    }
    for (int64_t p = beg + lane; p < end; p += G) {
      const uint32_t x = (uint32_t)adj[p];
#pragma unroll
      for (int j = 0; j < kKhBatch; ++j) {
        if (i0 + j < k) {
          const uint64_t key = mh_key(ha[i0 + j], hc[i0 + j], x);
          if (key < best[j] || (key == best[j] && x < bid[j])) {
            best[j] = key;
            bid[j] = x;
          }
        }
      }
    }
    if constexpr (G <= kWave) {
#pragma unroll
      for (int j = 0; j < kKhBatch; ++j) min_pair_group<G>(best[j], bid[j]);
    } else {
#pragma unroll
      for (int j = 0; j < kKhBatch; ++j) min_pair_group<kWave>(best[j], bid[j]);
      const int wv = threadIdx.x / kWave;
      if (lane_id() == 0) {
#pragma unroll
        for (int j = 0; j < kKhBatch; ++j) {
          lkey[wv * kKhBatch + j] = best[j];
          lid[wv * kKhBatch + j] = bid[j];
        }
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kKhBatch; ++j) {
        uint64_t bk = lkey[j];
        uint32_t bi = lid[j];
        for (int w = 1; w < kBlock / kWave; ++w) {
          const uint64_t ok = lkey[w * kKhBatch + j];
          const uint32_t oi = lid[w * kKhBatch + j];
          if (ok < bk || (ok == bk && oi < bi)) {
            bk = ok;
            bi = oi;
          }
        }
        best[j] = bk;
        bid[j] = bi;
      }
      __syncthreads();
    }
    if (active) {
      uint32_t* row = sig + (size_t)v * k;
#pragma unroll
      for (int j = 0; j < kKhBatch; ++j)
        if (i0 + j < k && (j % G) == lane) row[i0 + j] = bid[j];
    }
  }
}

// Heavy vertices (more than kMediumMax arcs), split into the work plan's
// chunks of kHeavyChunk arcs, one block per chunk: the chunk's argmin of every
// hash function, (key, element) per hash into the partials. One block per
// vertex let the largest hub set the length of the whole build.
__global__ __launch_bounds__(kBlock) void k_kh_build_chunks(PlanView P, const int32_t* __restrict__ adj, uint32_t k,
                                                            const uint64_t* __restrict__ ha,
                                                            const uint64_t* __restrict__ hc,
                                                            uint64_t* __restrict__ part_key,
                                                            uint32_t* __restrict__ part_id) {
  __shared__ uint64_t lkey[(kBlock / kWave) * kKhBatch];
  __shared__ uint32_t lid[(kBlock / kWave) * kKhBatch];
  const int64_t c = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t beg = P.chunk_begin[c], end = P.chunk_end[c];
  for (uint32_t i0 = 0; i0 < k; i0 += kKhBatch) {
    uint64_t best[kKhBatch];
    uint32_t bid[kKhBatch];
#pragma unroll
    for (int j = 0; j < kKhBatch; ++j) {
      best[j] = ~0ull;
      bid[j] = kBottom;
    }
    for (int64_t p = beg + tid; p < end; p += kBlock) {
      const uint32_t x = (uint32_t)adj[p];
#pragma unroll
      for (int j = 0; j < kKhBatch; ++j) {
        if (i0 + j < k) {
          const uint64_t key = mh_key(ha[i0 + j], hc[i0 + j], x);
          if (key < best[j] || (key == best[j] && x < bid[j])) {
            best[j] = key;
            bid[j] = x;
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kKhBatch; ++j) min_pair_group<kWave>(best[j], bid[j]);
    const int wv = tid / kWave;
    if (lane_id() == 0) {
#pragma unroll
      for (int j = 0; j < kKhBatch; ++j) {
        lkey[wv * kKhBatch + j] = best[j];
        lid[wv * kKhBatch + j] = bid[j];
      }
    }
    __syncthreads();
    if (tid < kKhBatch && i0 + tid < k) {
      uint64_t bk = lkey[tid];
      uint32_t bi = lid[tid];
      for (int w = 1; w < kBlock / kWave; ++w) {
        const uint64_t ok = lkey[w * kKhBatch + tid];
        const uint32_t oi = lid[w * kKhBatch + tid];
        if (ok < bk || (ok == bk && oi < bi)) {
          bk = ok;
          bi = oi;
        }
      }
      part_key[c * (int64_t)k + i0 + tid] = bk;
      part_id[c * (int64_t)k + i0 + tid] = bi;
    }
    __syncthreads();
  }
}

// Slot i of heavy vertex h: the least (key, element) over its chunks. The
// minimum does not depend on the order of the chunks.
__global__ void k_kh_combine(PlanView P, int64_t n_heavy, uint32_t k, const uint64_t* __restrict__ part_key,
                             const uint32_t* __restrict__ part_id, uint32_t* __restrict__ sig) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n_heavy * (int64_t)k) return;
  const int64_t h = t / k;
  const uint32_t i = (uint32_t)(t % k);
  const int32_t c0 = P.heavy_first[h], c1 = P.heavy_first[h + 1];
  uint64_t best = ~0ull;
  uint32_t bid = kBottom;
  for (int32_t c = c0; c < c1; ++c) {
    const uint64_t key = part_key[(int64_t)c * k + i];
    const uint32_t id = part_id[(int64_t)c * k + i];
    if (key < best || (key == best && id < bid)) {
      best = key;
      bid = id;
    }
  }
  sig[(size_t)P.chunk_vertex[c0] * k + i] = bid;
}

// ---------------------------------------------------------------- 1-hash

constexpr int kOhWaves = kBlock / kWave;

// Shared bytes per wave: k keys (8 B) + k IDs (4 B) + 256 histogram bins,
// rounded to 16 bytes so every wave's key array stays 8-byte aligned.
constexpr uint32_t kOhCand = 512;  // candidates of the k-th key's top-byte bin held in LDS
// Candidate slots per wave: kOhCand for k <= 512 (a block then needs at most
// 53 KB of LDS), none above.
__host__ __device__ constexpr uint32_t oh_cand(uint32_t k) { return k <= 512 ? kOhCand : 0u; }
__host__ __device__ constexpr size_t oh_wave_bytes(uint32_t k) {
  return (((size_t)k * 12 + 256 * 4 + (size_t)oh_cand(k) * 12) + 15) & ~(size_t)15;
}

// One wave per vertex. Shared memory per wave: keys and IDs of up to k
// elements, a 256-bin digit histogram, and kOhCand candidate keys and IDs.
// For d > k a radix select runs over the keys, 8 bits per pass from the top:
// each pass histograms the next byte of the keys that share the prefix found
// so far. As soon as the bin holding rank k has at most kOhCand keys, it
// splits N_v into the keys below the bin's prefix (all among the k smallest),
// the bin's keys and the rest: one more pass stages the first group and
// collects the bin in LDS, where the remaining smallest keys are found by
// rank counting. Every key is hashed twice when the first bin fits (d up to
// about 100,000), once more per further pass.
// The min(k, end - beg) elements of list[beg, end) with the smallest keys,
// in ascending key order, to row[0 ..), then kBottom up to row[k - 1]; run
// by one whole wave on its LDS slice.
__device__ void oh_select(const uint32_t* __restrict__ list, int64_t beg, int64_t end, uint32_t k, uint64_t a,
                          uint64_t c, uint32_t* __restrict__ row, unsigned char* __restrict__ slice) {
  const int lane = lane_id();
  // wave slice: [skey: k][ckey: cap] (8 bytes each), [sid: k][cid: cap][hist: 256] (4 bytes each)
  const uint32_t cap = oh_cand(k);
  uint64_t* skey = (uint64_t*)slice;
  uint64_t* ckey = skey + k;
  uint32_t* sid = (uint32_t*)(ckey + cap);
  uint32_t* cid = sid + k;
  uint32_t* hist = cid + cap;
  const int64_t d = end - beg;
  int64_t taken = 0;  // elements staged in skey/sid
  if (d <= (int64_t)k) {
    for (int64_t t = lane; t < d; t += kWave) {
      const uint32_t x = list[beg + t];
      skey[t] = mh_key(a, c, x);
      sid[t] = x;
    }
    taken = d;
  } else {
    // radix select of the k-th smallest key, 8 bits at a time from the top
    uint64_t prefix = 0, pmask = 0;
    uint32_t want = k;  // rank (1-based) still wanted among keys matching the prefix
    bool staged = false;
    for (int shift = 56; shift >= 0 && !staged; shift -= 8) {
      for (int i = lane; i < 256; i += kWave) hist[i] = 0;
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      for (int64_t t = beg + lane; t < end; t += kWave) {
        const uint64_t key = mh_key(a, c, list[t]);
        if ((key & pmask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      // find the digit holding rank `want`: lane l scans bins 4l..4l+3
      uint32_t local[4];
      uint32_t lsum = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        local[q] = hist[lane * 4 + q];
        lsum += local[q];
      }
      uint32_t incl = lsum;
#pragma unroll
      for (int dd = 1; dd < kWave; dd <<= 1) {
        const uint32_t y = __shfl_up(incl, dd);
        if (lane >= dd) incl += y;
      }
      const uint32_t excl = incl - lsum;
      int digit = -1;
      uint32_t below = 0;
      if (excl < want && want <= incl) {
        uint32_t run = excl;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (digit < 0 && want <= run + local[q]) {
            digit = lane * 4 + q;
            below = run;
          }
          run += local[q];
        }
      }
      const unsigned long long owner = __ballot(digit >= 0);
      const int src = __ffsll((long long)owner) - 1;
      digit = __shfl(digit, src);
      below = __shfl(below, src);
      const uint32_t nc = hist[digit];  // keys in the bin holding rank `want`
      if (nc <= cap) {
        // one pass: the keys below the bin's prefix P (k - want + below of
        // them, all among the k smallest) go straight to skey, the bin's keys
        // to the candidates
        const uint64_t P = prefix | ((uint64_t)digit << shift);
        const uint64_t M = pmask | (255ull << shift);
        const uint32_t nbelow = k - want + below;
        uint32_t nlo = 0, ncand = 0;
        const uint64_t lanes_before = (1ull << lane) - 1ull;
        for (int64_t t0 = beg; t0 < end; t0 += kWave) {
          const int64_t t = t0 + lane;
          uint64_t key = 0;
          uint32_t x = 0;
          if (t < end) {
            x = list[t];
            key = mh_key(a, c, x);
          }
          const bool lo = t < end && key < P;
          const bool in_bin = t < end && (key & M) == P;
          const unsigned long long blo = __ballot(lo), bin = __ballot(in_bin);
          if (lo) {
            const uint32_t pos = nlo + (uint32_t)__popcll(blo & lanes_before);
            skey[pos] = key;
            sid[pos] = x;
          }
          if (in_bin) {
            const uint32_t pos = ncand + (uint32_t)__popcll(bin & lanes_before);
            ckey[pos] = key;
            cid[pos] = x;
          }
          nlo += (uint32_t)__popcll(blo);
          ncand += (uint32_t)__popcll(bin);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // the want smallest candidates complete the k smallest (keys distinct)
        for (uint32_t t = (uint32_t)lane; t < nc; t += kWave) {
          const uint64_t key = ckey[t];
          uint32_t r = 0;
          for (uint32_t q = 0; q < nc; ++q) r += ckey[q] < key ? 1u : 0u;
          if (r < want - below) {
            skey[nbelow + r] = key;
            sid[nbelow + r] = cid[t];
          }
        }
        staged = true;
        break;
      }
      prefix |= (uint64_t)digit << shift;
      pmask |= 255ull << shift;
      want -= below;
    }
    // prefix is now the k-th smallest key: stage the k keys <= prefix
    int64_t base = 0;
    for (int64_t t0 = staged ? end : beg; t0 < end; t0 += kWave) {
      const int64_t t = t0 + lane;
      uint64_t key = 0;
      uint32_t x = 0;
      bool keep = false;
      if (t < end) {
        x = list[t];
        key = mh_key(a, c, x);
        keep = key <= prefix;
      }
      const unsigned long long bal = __ballot(keep);
      if (keep) {
        const int64_t pos = base + __popcll(bal & ((1ull << lane) - 1ull));
        if (pos < (int64_t)k) {  // exactly k keys qualify when the IDs of N_v are distinct
          skey[pos] = key;
          sid[pos] = x;
        }
      }
      base += __popcll(bal);
    }
    taken = staged ? (int64_t)k : (base < (int64_t)k ? base : (int64_t)k);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  // rank sort of the staged elements (keys distinct)
  for (int64_t t = lane; t < taken; t += kWave) {
    const uint64_t key = skey[t];
    uint32_t r = 0;
    for (int64_t q = 0; q < taken; ++q) r += skey[q] < key ? 1u : 0u;
    row[r] = sid[t];
  }
  for (int64_t t = taken + lane; t < (int64_t)k; t += kWave) row[t] = kBottom;
}

__device__ __forceinline__ unsigned char* oh_slice(uint32_t k) {
  extern __shared__ unsigned char smem[];
  return smem + (threadIdx.x / kWave) * oh_wave_bytes(k);
}

// One wave per listed vertex; vertices of more than max_deg arcs are left to
// the chunk kernels.
__global__ __launch_bounds__(kBlock) void k_oh_build(const int32_t* __restrict__ off, const int32_t* __restrict__ adj,
                                                     const int32_t* __restrict__ verts, int64_t nverts, uint32_t k,
                                                     uint64_t a, uint64_t c, uint32_t* __restrict__ sig,
                                                     int64_t max_deg) {
  const int64_t grp = blockIdx.x * (int64_t)kOhWaves + threadIdx.x / kWave;
  if (grp >= nverts) return;
  const int32_t v = verts[grp];
  const int64_t beg = off[v], end = off[v + 1];
  if (end - beg > max_deg) return;
  oh_select(reinterpret_cast<const uint32_t*>(adj), beg, end, k, a, c, sig + (size_t)v * k, oh_slice(k));
}

// Heavy vertices: one wave per work-plan chunk writes the chunk's smallest
// min(k, arcs) elements to cand[chunk * k ..]; then one wave per heavy vertex
// selects the k smallest among its chunks' candidates, which hold them (the
// k smallest of a union are among the k smallest of each part). Every chunk
// but a vertex's last has kHeavyChunk >= k arcs, so a vertex's candidates are
// contiguous.
__global__ __launch_bounds__(kBlock) void k_oh_build_chunks(PlanView P, const int32_t* __restrict__ adj, uint32_t k,
                                                            uint64_t a, uint64_t c, uint32_t* __restrict__ cand) {
  const int64_t ch = blockIdx.x * (int64_t)kOhWaves + threadIdx.x / kWave;
  if (ch >= P.n_chunks) return;
  oh_select(reinterpret_cast<const uint32_t*>(adj), P.chunk_begin[ch], P.chunk_end[ch], k, a, c, cand + (size_t)ch * k,
            oh_slice(k));
}

__global__ __launch_bounds__(kBlock) void k_oh_build_combine(PlanView P, int64_t n_heavy,
                                                             const uint32_t* __restrict__ cand, uint32_t k, uint64_t a,
                                                             uint64_t c, uint32_t* __restrict__ sig) {
  const int64_t h = blockIdx.x * (int64_t)kOhWaves + threadIdx.x / kWave;
  if (h >= n_heavy) return;
  const int32_t c0 = P.heavy_first[h], c1 = P.heavy_first[h + 1];
  const int64_t last = P.chunk_end[c1 - 1] - P.chunk_begin[c1 - 1];
  const int64_t end = (int64_t)(c1 - 1) * k + (last < (int64_t)k ? last : (int64_t)k);
  oh_select(cand, (int64_t)c0 * k, end, k, a, c, sig + (size_t)P.chunk_vertex[c0] * k, oh_slice(k));
}

// Vertices of at most D arcs (and k >= D): every element is kept, so the row
// is N_v in ascending key order, then kBottom. G lanes per vertex hash its
// elements into the group's LDS slice, rank them (keys are distinct) and
// write the row in 16-byte pieces when k is a multiple of 4. A wave per such
// small vertex spent most of its time starting and finishing (R-MAT s24,
// k = 64: 21.6 -> 17.5 ms for the whole build; a second tier of 16 lanes for
// 17..64 arcs changed nothing, the radix selection of the larger vertices
// takes the rest).
constexpr int kOhSmall = 16;  // degree bin 0: 4 lanes per vertex

template <int G, int D>
__global__ __launch_bounds__(kBlock) void k_oh_build_small(const int32_t* __restrict__ off,
                                                           const int32_t* __restrict__ adj,
                                                           const int32_t* __restrict__ verts, int64_t nverts,
                                                           uint32_t k, uint64_t a, uint64_t c,
                                                           uint32_t* __restrict__ sig) {
  static_assert(kWave % G == 0, "groups lie inside one wave");
  __shared__ uint64_t skey[kBlock / G][D];
  __shared__ uint32_t sid[kBlock / G][D];
  __shared__ uint32_t sorted[kBlock / G][D];
  const int grp = threadIdx.x / G;
  const int lane = threadIdx.x % G;
  const int64_t gi = blockIdx.x * (int64_t)(kBlock / G) + grp;
  const int32_t v = gi < nverts ? verts[gi] : 0;
  const int64_t beg = gi < nverts ? off[v] : 0;
  const int64_t dv = gi < nverts ? off[v + 1] - beg : 0;
  const bool active = gi < nverts && dv <= D;
  const int d = active ? (int)dv : 0;
  for (int t = lane; t < d; t += G) {
    const uint32_t x = (uint32_t)adj[beg + t];
    skey[grp][t] = mh_key(a, c, x);
    sid[grp][t] = x;
  }
  wave_sync();
  for (int t = lane; t < d; t += G) {
    const uint64_t key = skey[grp][t];
    int r = 0;
    for (int q = 0; q < d; ++q) r += skey[grp][q] < key ? 1 : 0;
    sorted[grp][r] = sid[grp][t];
  }
  wave_sync();
  if (!active) return;
  uint32_t* row = sig + (size_t)v * k;
  if (k % 4 == 0) {
    uint4* row4 = reinterpret_cast<uint4*>(row);
    for (uint32_t q = (uint32_t)lane; q < k / 4; q += G) {
      uint32_t e[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t i = 4 * q + (uint32_t)j;
        e[j] = i < (uint32_t)d ? sorted[grp][i] : kBottom;
      }
      row4[q] = make_uint4(e[0], e[1], e[2], e[3]);
    }
  } else {
    for (uint32_t i = (uint32_t)lane; i < k; i += G) row[i] = i < (uint32_t)d ? sorted[grp][i] : kBottom;
  }
}

// Dense copy of the rows (row v at v * W words) for export.
__global__ void k_bf_unpack(const uint64_t* __restrict__ words, int64_t n, uint32_t W, uint64_t* __restrict__ out) {
  const int64_t total = n * (int64_t)W;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = i / W;
    out[i] = words[bf_row_offset(v, W) + (i - v * W)];
  }
}

// Line-packed rows from a dense copy (row v at v * W words).
__global__ void k_bf_pack(const uint64_t* __restrict__ dense, int64_t n, uint32_t W, uint64_t* __restrict__ words) {
  const int64_t total = n * (int64_t)W;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = i / W;
    words[bf_row_offset(v, W) + (i - v * W)] = dense[i];
  }
}

// Ones of each dense row.
__global__ void k_bf_popcounts(const uint64_t* __restrict__ dense, int64_t n, uint32_t W, uint32_t* __restrict__ pc) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    uint32_t ones = 0;
    for (uint32_t k = 0; k < W; ++k) ones += (uint32_t)__popcll(dense[v * W + k]);
    pc[v] = ones;
  }
}

// Number of i with a[i] != b[i], added to *bad.
__global__ void k_u32_mismatches(const uint32_t* __restrict__ a, const uint32_t* __restrict__ b, int64_t n,
                                 unsigned long long* __restrict__ bad) {
  uint32_t mine = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    mine += a[i] != b[i] ? 1u : 0u;
  if (mine) atomicAdd(bad, (unsigned long long)mine);
}

}  // namespace

int bf_pack(pg_sketches* sk, const void* rows, const uint32_t* pc, hipStream_t s) {
  const int64_t n = sk->rows->n;
  sk->empty_rows_zero = false;  // the next build writes every row again
  if (n <= 0) return PG_OK;
  hipLaunchKernelGGL(k_bf_pack, dim3(grid_for(n * sk->W, kBlock, 65536)), dim3(kBlock), 0, s,
                     (const uint64_t*)rows, n, sk->W, sk->words);
  PG_LAUNCH_CHECK();
  // the popcounts are always counted from the rows: the OR estimator indexes
  // its table of B + 1 entries with pc_u + pc_v - c, so a count that is not
  // the row's could read past it
  hipLaunchKernelGGL(k_bf_popcounts, dim3(grid_for(n, kBlock, 65536)), dim3(kBlock), 0, s, (const uint64_t*)rows, n,
                     sk->W, sk->pc);
  PG_LAUNCH_CHECK();
  if (!pc) return PG_OK;
  // given popcounts must equal the counted ones
  unsigned long long* d_bad = nullptr;
  PG_TRY(dmalloc((void**)&d_bad, sizeof(unsigned long long), s));
  int rc = fill_u64((uint64_t*)d_bad, 0, 1, s);
  if (rc == PG_OK) {
    hipLaunchKernelGGL(k_u32_mismatches, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, s, pc,
                       (const uint32_t*)sk->pc, n, d_bad);
    if (hipGetLastError() != hipSuccess) rc = fail(PG_E_DEVICE, "popcount check launch failed");
  }
  unsigned long long bad = 0;
  if (rc == PG_OK) {
    hipError_t e = hipMemcpyAsync(&bad, d_bad, sizeof(bad), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = fail(PG_E_DEVICE, std::string("popcount check: ") + hipGetErrorString(e));
  }
  dfree(d_bad, s);
  if (rc == PG_OK && bad)
    rc = fail(PG_E_INVALID, std::to_string(bad) + " given popcounts differ from the ones of their rows");
  return rc;
}

int bf_unpack(const pg_sketches* sk, void* rows, hipStream_t s) {
  const int64_t n = sk->rows->n;
  if (n <= 0) return PG_OK;
  hipLaunchKernelGGL(k_bf_unpack, dim3(grid_for(n * sk->W, kBlock, 65536)), dim3(kBlock), 0, s,
                     (const uint64_t*)sk->words, n, sk->W, (uint64_t*)rows);
  PG_LAUNCH_CHECK();
  return PG_OK;
}

int build_bf(pg_sketches* sk, hipStream_t s) {
  const pg_graph* g = sk->rows;  // the lists the rows sketch (N_v or N+_v)
  ProfScope ps(s, "bf_build");
  const uint32_t W = sk->W;
  if (W <= 16 && g->n > 0) {
    const VertexPlan& P = g->plan_all;
    PlanView pv = plan_view(P);
    // the rows of vertices without arcs (the tail of the light list) are
    // zero under every seed: once written, later builds leave them
    if (sk->empty_rows_zero) pv.n_light -= P.n_empty;
    const unsigned grid = (unsigned)(P.n_chunks + pv.n_medium_blocks + (pv.n_light * kLightGroup + kBlock - 1) / kBlock);
    if (grid == 0) return PG_OK;  // every vertex without arcs, rows already zero
    const unsigned cgrid = (unsigned)((P.n_heavy * kWave + kBlock - 1) / kBlock);
#define PG_BFP(WW)                                                                                                 \
  do {                                                                                                             \
    hipLaunchKernelGGL((k_bf_build_plan<WW>), dim3(grid), dim3(kBlock), 0, s, pv, g->off, g->adj, sk->size, sk->b, \
                       sk->ha, sk->hc, sk->words, sk->pc, sk->scratch);                                            \
    if (P.n_heavy > 0)                                                                                             \
      hipLaunchKernelGGL((k_bf_combine<WW>), dim3(cgrid), dim3(kBlock), 0, s, pv, (const uint64_t*)sk->scratch,    \
                         P.n_heavy, sk->words, sk->pc);                                                            \
  } while (0)
    switch (W) {
      case 1: PG_BFP(1); break;
      case 2: PG_BFP(2); break;
      case 3: PG_BFP(3); break;
      case 4: PG_BFP(4); break;
      case 5: PG_BFP(5); break;
      case 6: PG_BFP(6); break;
      case 7: PG_BFP(7); break;
      case 8: PG_BFP(8); break;
      case 9: PG_BFP(9); break;
      case 10: PG_BFP(10); break;
      case 11: PG_BFP(11); break;
      case 12: PG_BFP(12); break;
      case 13: PG_BFP(13); break;
      case 14: PG_BFP(14); break;
      case 15: PG_BFP(15); break;
      default: PG_BFP(16); break;
    }
#undef PG_BFP
    PG_LAUNCH_CHECK();
    sk->empty_rows_zero = true;
    return PG_OK;
  }
  if (g->n > 0) {  // filters wider than 16 words
    hipLaunchKernelGGL(k_bf_build_wide, dim3(grid_for((int64_t)g->n * kWave, kBlock, 1ll << 31)), dim3(kBlock), 0, s,
                       g->off, g->adj, g->n, sk->size, W, sk->b, sk->ha, sk->hc, sk->words, sk->pc);
    PG_LAUNCH_CHECK();
  }
  return PG_OK;
}

int build_khash(pg_sketches* sk, hipStream_t s) {
  const pg_graph* g = sk->rows;  // the lists the rows sketch (N_v or N+_v)
  ProfScope ps(s, "kh_build");
  const VertexPlan& P = g->plan_all;
  // vertices up to kMediumMax arcs by degree bin; the heavier ones in chunks
  for (int bin = 0; bin < kNumBins; ++bin) {
    const int64_t cnt = g->bin_start[bin + 1] - g->bin_start[bin];
    if (cnt <= 0) continue;
    if (bin > 0 && kBinMaxDeg[bin - 1] >= kMediumMax) continue;  // every vertex of the bin is heavy
    const int32_t* verts = g->bin_verts + g->bin_start[bin];
    const int G = std::min(kBinGroup[bin], kWave);
    const unsigned grid = (unsigned)((cnt * G + kBlock - 1) / kBlock);
    const int64_t max_deg = kMediumMax;
    if (G == 4)
      hipLaunchKernelGGL(k_kh_build<4>, dim3(grid), dim3(kBlock), 0, s, g->off, g->adj, verts, cnt, sk->size, sk->ha,
                         sk->hc, sk->sig, max_deg);
    else if (G == 16)
      hipLaunchKernelGGL(k_kh_build<16>, dim3(grid), dim3(kBlock), 0, s, g->off, g->adj, verts, cnt, sk->size, sk->ha,
                         sk->hc, sk->sig, max_deg);
    else
      hipLaunchKernelGGL(k_kh_build<64>, dim3(grid), dim3(kBlock), 0, s, g->off, g->adj, verts, cnt, sk->size, sk->ha,
                         sk->hc, sk->sig, max_deg);
    PG_LAUNCH_CHECK();
  }
  if (P.n_chunks > 0) {
    const PlanView pv = plan_view(P);
    uint64_t* part_key = sk->scratch;
    uint32_t* part_id = reinterpret_cast<uint32_t*>(sk->scratch + P.n_chunks * (int64_t)sk->size);
    hipLaunchKernelGGL(k_kh_build_chunks, dim3((unsigned)P.n_chunks), dim3(kBlock), 0, s, pv, g->adj, sk->size, sk->ha,
                       sk->hc, part_key, part_id);
    PG_LAUNCH_CHECK();
    const int64_t t = P.n_heavy * (int64_t)sk->size;
    hipLaunchKernelGGL(k_kh_combine, dim3((unsigned)((t + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, pv, P.n_heavy,
                       sk->size, (const uint64_t*)part_key, (const uint32_t*)part_id, sk->sig);
    PG_LAUNCH_CHECK();
  }
  return PG_OK;
}

int build_onehash(pg_sketches* sk, hipStream_t s) {
  const pg_graph* g = sk->rows;  // the lists the rows sketch (N_v or N+_v)
  const int64_t nv = g->n;
  if (nv <= 0) return PG_OK;
  const size_t shmem = (size_t)kOhWaves * oh_wave_bytes(sk->size);
  uint64_t a = 0, c = 0;
  hash_constants(PG_MH_1HASH, sk->seed, 1, &a, &c);
  ProfScope ps(s, "oh_build");
  // vertices of at most kOhSmall arcs (degree bin 0) four lanes each, the
  // others a wave each, in bin order (degree-sorted blocks balance better)
  static_assert(kBinMaxDeg[0] == kOhSmall, "bin 0 holds the small vertices");
  const int64_t n0 = sk->size >= (uint32_t)kOhSmall ? g->bin_start[1] - g->bin_start[0] : 0;
  if (n0 > 0) {
    constexpr int G = 4;
    hipLaunchKernelGGL((k_oh_build_small<G, kOhSmall>), dim3((unsigned)((n0 * G + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, g->off, g->adj, g->bin_verts, n0, sk->size, a, c, sk->sig);
    PG_LAUNCH_CHECK();
  }
  // heavy vertices in the work plan's chunks when k fits a chunk (the scratch
  // then holds k candidates per chunk)
  const VertexPlan& P = g->plan_all;
  const bool chunked = P.n_chunks > 0 && sk->size <= (uint32_t)kHeavyChunk && sk->scratch;
  if (nv - n0 > 0) {
    hipLaunchKernelGGL(k_oh_build, dim3((unsigned)((nv - n0 + kOhWaves - 1) / kOhWaves)), dim3(kBlock), shmem, s,
                       g->off, g->adj, g->bin_verts + n0, nv - n0, sk->size, a, c, sk->sig,
                       chunked ? (int64_t)kMediumMax : INT64_MAX);
    PG_LAUNCH_CHECK();
  }
  if (chunked) {
    const PlanView pv = plan_view(P);
    uint32_t* cand = reinterpret_cast<uint32_t*>(sk->scratch);
    hipLaunchKernelGGL(k_oh_build_chunks, dim3((unsigned)((P.n_chunks + kOhWaves - 1) / kOhWaves)), dim3(kBlock),
                       shmem, s, pv, g->adj, sk->size, a, c, cand);
    PG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_oh_build_combine, dim3((unsigned)((P.n_heavy + kOhWaves - 1) / kOhWaves)), dim3(kBlock),
                       shmem, s, pv, P.n_heavy, (const uint32_t*)cand, sk->size, a, c, sk->sig);
    PG_LAUNCH_CHECK();
  }
  return PG_OK;
}

}  // namespace pg
