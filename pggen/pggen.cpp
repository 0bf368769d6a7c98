// Seeded synthetic graph generator: R-MAT and Erdos-Renyi G(n,p), emitted as a
// symmetric, sorted, duplicate-free, self-loop-free CSR with int32 offsets and
// int32 neighbour IDs (the storage layout of the paper's Section 2.1: all
// neighbourhoods in one contiguous sorted array plus an offsets array).
//
// This module produces inputs only. It holds none of the method's arithmetic
// (no sketch, hash or estimator) and is shared by the test oracle and by the
// GPU library's tests and benchmark, which feed it identical bytes.
//
// Random numbers come from SplitMix64 (Steele, Lea, Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014) used as a counter-based
// generator: output i of the stream keyed by s is mix(s + (i+1)*gamma).
//
// R-MAT follows Chakrabarti, Zhan, Faloutsos (SDM 2004): every edge descends
// `scale` levels of the 2x2 recursive matrix, choosing a quadrant with
// probabilities (a, b, c, d) at each level. The paper's synthetic family is
// the Kronecker power-law model (Section 8.1); R-MAT is its 2x2 stochastic
// instance. G(n,p) uses geometric skipping over the linear pair index
// (Batagelj and Brandes, Phys. Rev. E 71, 2005).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Output i (0-based) of the SplitMix64 stream whose initial state is `key`.
inline uint64_t stream_at(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * kGamma); }

// Domain tags keep the R-MAT and ER streams of one seed apart.
constexpr uint64_t kTagRmat = 0x524D4154ull;  // "RMAT"
constexpr uint64_t kTagEr = 0x45524E50ull;    // "ERNP"

struct RmatThresholds {
  uint64_t ta, tab, tabc;
};

inline void rmat_draw(uint64_t key, uint64_t attempt, int scale, const RmatThresholds& t,
                      uint32_t* src, uint32_t* dst) {
  uint32_t s = 0, d = 0;
  for (int l = 0; l < scale; ++l) {
    const uint64_t r = stream_at(key, attempt * (uint64_t)scale + (uint64_t)l) >> 11;  // 53 bits
    const uint32_t bit = 1u << (scale - 1 - l);
    if (r < t.ta) {
      // top-left quadrant: neither bit set
    } else if (r < t.tab) {
      d |= bit;
    } else if (r < t.tabc) {
      s |= bit;
    } else {
      s |= bit;
      d |= bit;
    }
  }
  *src = s;
  *dst = d;
}

}  // namespace

extern "C" {

// Output i of the SplitMix64 stream with initial state `key` (exported so the
// tests can check the generator against the published SplitMix64 vectors).
uint64_t pggen_splitmix64(uint64_t key, uint64_t i) { return stream_at(key, i); }

// R-MAT edge draws. n is the vertex count; scale = ceil(log2 n). When n is a
// power of two every draw is kept and draw e uses counter block e; otherwise
// draws with an endpoint >= n are rejected and redrawn from the next counter
// block, in sequence. Writes npairs (src, dst) pairs. Returns 0, or -1 on bad
// arguments.
int pggen_rmat_pairs(int32_t n, int64_t npairs, double a, double b, double c, uint64_t seed,
                     int32_t* src, int32_t* dst) {
  if (n < 1 || npairs < 0 || !src || !dst) return -1;
  if (a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return -1;
  int scale = 0;
  while ((int64_t(1) << scale) < (int64_t)n) ++scale;
  const double two53 = 9007199254740992.0;
  RmatThresholds t{(uint64_t)std::floor(a * two53), (uint64_t)std::floor((a + b) * two53),
                   (uint64_t)std::floor((a + b + c) * two53)};
  const uint64_t key = seed ^ kTagRmat;
  const bool pow2 = (int64_t(1) << scale) == (int64_t)n;
  if (scale == 0) {
    for (int64_t e = 0; e < npairs; ++e) src[e] = dst[e] = 0;
    return 0;
  }
  if (pow2) {
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < npairs; ++e) {
      uint32_t s, d;
      rmat_draw(key, (uint64_t)e, scale, t, &s, &d);
      src[e] = (int32_t)s;
      dst[e] = (int32_t)d;
    }
  } else {
    uint64_t attempt = 0;
    for (int64_t e = 0; e < npairs;) {
      uint32_t s, d;
      rmat_draw(key, attempt++, scale, t, &s, &d);
      if (s < (uint32_t)n && d < (uint32_t)n) {
        src[e] = (int32_t)s;
        dst[e] = (int32_t)d;
        ++e;
      }
    }
  }
  return 0;
}

// G(n,p) by geometric skipping over the pairs (v, w), w < v, in the order
// (1,0), (2,0), (2,1), (3,0), ... . With src == NULL only counts. Returns the
// number of pairs (at most cap are written), or -1 on bad arguments.
int64_t pggen_er_pairs(int32_t n, double p, uint64_t seed, int32_t* src, int32_t* dst, int64_t cap) {
  if (n < 1 || !(p >= 0.0) || p > 1.0) return -1;
  if (p == 0.0 || n < 2) return 0;
  const uint64_t key = seed ^ kTagEr;
  int64_t count = 0;
  if (p == 1.0) {
    for (int64_t v = 1; v < n; ++v)
      for (int64_t w = 0; w < v; ++w) {
        if (src && count < cap) {
          src[count] = (int32_t)v;
          dst[count] = (int32_t)w;
        }
        ++count;
      }
    return count;
  }
  const double lq = std::log(1.0 - p);
  int64_t v = 1, w = -1;
  uint64_t j = 0;
  while (v < n) {
    const double r = (double)(stream_at(key, j++) >> 11) * (1.0 / 9007199254740992.0);  // [0,1)
    w += 1 + (int64_t)std::floor(std::log(1.0 - r) / lq);
    while (w >= v && v < n) {
      w -= v;
      ++v;
    }
    if (v < n) {
      if (src && count < cap) {
        src[count] = (int32_t)v;
        dst[count] = (int32_t)w;
      }
      ++count;
    }
  }
  return count;
}

// Undirected CSR from a list of pairs: both directions are added, self-loops
// dropped, each neighbourhood sorted ascending and deduplicated. offsets has
// n+1 entries; adj has room for cap IDs. Returns nnz, -1 on bad arguments, or
// -2 when nnz would exceed cap or INT32_MAX.
int64_t pggen_csr_build(int32_t n, int64_t npairs, const int32_t* src, const int32_t* dst,
                        int32_t* offsets, int32_t* adj, int64_t cap) {
  if (n < 0 || npairs < 0 || !offsets || (npairs > 0 && (!src || !dst))) return -1;
  std::vector<int64_t> start((size_t)n + 1, 0);
  for (int64_t e = 0; e < npairs; ++e) {
    const int32_t s = src[e], d = dst[e];
    if (s < 0 || d < 0 || s >= n || d >= n) return -1;
    if (s == d) continue;
    ++start[(size_t)s + 1];
    ++start[(size_t)d + 1];
  }
  for (int32_t v = 0; v < n; ++v) start[(size_t)v + 1] += start[v];
  const int64_t total = start[n];
  std::vector<int32_t> tmp((size_t)total);
  {
    std::vector<int64_t> pos(start.begin(), start.end() - 1);
    for (int64_t e = 0; e < npairs; ++e) {
      const int32_t s = src[e], d = dst[e];
      if (s == d) continue;
      tmp[(size_t)pos[s]++] = d;
      tmp[(size_t)pos[d]++] = s;
    }
  }
  std::vector<int64_t> len((size_t)n, 0);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t v = 0; v < n; ++v) {
    int32_t* b = tmp.data() + start[v];
    int32_t* e = tmp.data() + start[(size_t)v + 1];
    std::sort(b, e);
    len[v] = std::unique(b, e) - b;
  }
  int64_t nnz = 0;
  for (int32_t v = 0; v < n; ++v) nnz += len[v];
  if (nnz > cap || nnz > (int64_t)INT32_MAX) return -2;
  int64_t o = 0;
  for (int32_t v = 0; v < n; ++v) {
    offsets[v] = (int32_t)o;
    if (adj) std::memcpy(adj + o, tmp.data() + start[v], (size_t)len[v] * sizeof(int32_t));
    o += len[v];
  }
  offsets[n] = (int32_t)o;
  return nnz;
}

}  // extern "C"
