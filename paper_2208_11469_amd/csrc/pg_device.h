// Device-side helpers shared by the library's kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pg {

constexpr uint32_t kBottom = 0xFFFFFFFFu;  // empty MinHash slot
constexpr int kWave = 64;

// SplitMix64's output mix (Steele, Lea, Flood 2014): a bijection of 64-bit words.
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Bloom-filter bit of element x under hash (a, c): the top 32 bits of the
// multiply-add a*x + c (mod 2^64), scaled to [0, B) by a multiply-high.
__device__ __forceinline__ uint32_t bf_index(uint64_t a, uint64_t c, uint32_t x, uint32_t B) {
  const uint64_t g = a * (uint64_t)x + c;
  return __umulhi((uint32_t)(g >> 32), B);
}

// MinHash key of element x under hash (a, c): mix64(a*x + c). Odd a makes the
// map injective on 64-bit words, so different vertices never tie.
__device__ __forceinline__ uint64_t mh_key(uint64_t a, uint64_t c, uint32_t x) {
  return mix64(a * (uint64_t)x + c);
}

// Bloom-filter row layout ("line-packed"): rows of W 64-bit words are packed
// r = bf_rows_per_group(W) to a group of bf_group_words(W) words. For the
// widths where a 128-byte group wastes at most a quarter of its bytes, groups
// are exactly 128 bytes, so no row crosses a 128-byte cache line and a row
// gather touches one line; other widths stay dense (r = 1, group = W).
__host__ __device__ constexpr uint32_t bf_rows_per_group(uint32_t W) {
  return (W <= 16 && 16 % W <= 4) ? 16 / W : 1;
}
__host__ __device__ constexpr uint32_t bf_group_words(uint32_t W) { return (W <= 16 && 16 % W <= 4) ? 16 : W; }
__host__ __device__ __forceinline__ size_t bf_row_offset(int64_t v, uint32_t W) {
  const uint32_t r = bf_rows_per_group(W);
  return (size_t)(v / r) * bf_group_words(W) + (size_t)(v % r) * W;
}
// Words of a sketch set of n rows.
__host__ __device__ constexpr size_t bf_total_words(int64_t n, uint32_t W) {
  return (size_t)((n + bf_rows_per_group(W) - 1) / bf_rows_per_group(W)) * bf_group_words(W);
}
// Slack words allocated after the last group: team readers of a row may read
// up to 15 words past its end (those words are never counted).
constexpr size_t kBfSlackWords = 16;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Fixed-order butterfly sum over groups of G lanes (G a power of two <= 64);
// every lane of the group ends with the same bits.
template <int G>
__device__ __forceinline__ double group_sum(double x) {
#pragma unroll
  for (int s = G / 2; s >= 1; s >>= 1) x += __shfl_xor(x, s, G);
  return x;
}

template <int G>
__device__ __forceinline__ uint64_t group_or(uint64_t x) {
#pragma unroll
  for (int s = G / 2; s >= 1; s >>= 1) x |= __shfl_xor(x, s, G);
  return x;
}

template <int G>
__device__ __forceinline__ uint64_t group_min(uint64_t x) {
#pragma unroll
  for (int s = G / 2; s >= 1; s >>= 1) {
    const uint64_t y = __shfl_xor(x, s, G);
    x = y < x ? y : x;
  }
  return x;
}

template <int G>
__device__ __forceinline__ uint32_t group_sum_u32(uint32_t x) {
#pragma unroll
  for (int s = G / 2; s >= 1; s >>= 1) x += __shfl_xor(x, s, G);
  return x;
}

// Sum over the T lanes of a team (T in {1, 2, 4}, teams aligned to quads) by
// quad DPP moves; every lane of the team ends with the sum. The lanes of a team
// must be active together.
template <int T>
__device__ __forceinline__ uint32_t team_sum(uint32_t c) {
  if constexpr (T >= 2) c += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)c, 0xB1, 0xF, 0xF, false);  // lane ^ 1
  if constexpr (T >= 4) c += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)c, 0x4E, 0xF, 0xF, false);  // lane ^ 2
  return c;
}

// Block-wide deterministic FP64 sum for blockDim.x == 256 (4 waves); result
// valid in thread 0.
__device__ __forceinline__ double block_sum_256(double x, double* lds4) {
  x = group_sum<64>(x);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds4[w] = x;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = ((lds4[0] + lds4[1]) + (lds4[2] + lds4[3]));
  __syncthreads();
  return r;
}

}  // namespace pg
