/* Test driver: runs every routine of the oracle's C half (oracle/pg_oracle.c)
 * over one graph read from a file, so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer checks their memory accesses and arithmetic.
 * File: int32 n, int64 nnz, int32 off[n+1], int32 adj[nnz], int64 m,
 * int32 poff[n+1], int32 padj[m] (degree-oriented lists), int32 deg[n].
 * Prints the counts the test compares against the regular oracle build. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t or_upper_edges(int32_t n, const int32_t* off, const int32_t* adj, int32_t* eu, int32_t* ev);
void or_exact_pairs(int32_t n, const int32_t* off, const int32_t* adj, int64_t npairs, const int32_t* pu,
                    const int32_t* pv, uint32_t* out);
uint64_t or_exact_tc_listing(int32_t n, const int32_t* off, const int32_t* adj);
uint64_t or_four_cliques(int32_t n, const int32_t* poff, const int32_t* padj, const int32_t* deg,
                         const uint64_t* words, uint32_t B, uint32_t b, uint64_t seed);
void or_four_cliques_filters(int32_t n, const int32_t* poff, const int32_t* padj, const uint64_t* words, uint32_t B,
                             uint32_t b, uint64_t seed, uint64_t* hist_and, uint64_t* hist_or, uint64_t* sizes);
void or_bf_build(int32_t n, const int32_t* off, const int32_t* adj, uint32_t B, uint32_t b, uint64_t seed,
                 uint64_t* words, uint32_t* pc);
void or_bf_counts(uint32_t W, const uint64_t* words, int64_t npairs, const int32_t* pu, const int32_t* pv,
                  uint32_t* c_and, uint32_t* c_or);
void or_kh_build(int32_t n, const int32_t* off, const int32_t* adj, uint32_t k, uint64_t seed, uint32_t* sig);
void or_kh_counts(uint32_t k, const uint32_t* sig, int64_t npairs, const int32_t* pu, const int32_t* pv,
                  uint32_t* s);
void or_1h_build(int32_t n, const int32_t* off, const int32_t* adj, uint32_t k, uint64_t seed, uint32_t* sig);
void or_1h_counts(uint32_t k, uint64_t seed, const uint32_t* sig, int64_t npairs, const int32_t* pu,
                  const int32_t* pv, uint32_t* s_uni, uint32_t* kprime, uint32_t* s_lit);

static void* xread(FILE* f, size_t bytes) {
  void* p = malloc(bytes > 0 ? bytes : 1);
  if (!p || fread(p, 1, bytes, f) != bytes) exit(2);
  return p;
}

static uint64_t sum32(const uint32_t* x, int64_t n) {
  uint64_t s = 0;
  for (int64_t i = 0; i < n; ++i) s += x[i];
  return s;
}

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t n;
  int64_t nnz, m_file;
  if (fread(&n, sizeof n, 1, f) != 1 || fread(&nnz, sizeof nnz, 1, f) != 1) return 2;
  int32_t* off = xread(f, sizeof(int32_t) * ((size_t)n + 1));
  int32_t* adj = xread(f, sizeof(int32_t) * (size_t)nnz);
  if (fread(&m_file, sizeof m_file, 1, f) != 1) return 2;
  int32_t* poff = xread(f, sizeof(int32_t) * ((size_t)n + 1));
  int32_t* padj = xread(f, sizeof(int32_t) * (size_t)m_file);
  int32_t* deg = xread(f, sizeof(int32_t) * (size_t)n);
  fclose(f);

  const int64_t m = or_upper_edges(n, off, adj, NULL, NULL);
  int32_t* eu = malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  int32_t* ev = malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  or_upper_edges(n, off, adj, eu, ev);
  uint32_t* a = malloc(sizeof(uint32_t) * (size_t)(m > 0 ? m : 1));
  uint32_t* b = malloc(sizeof(uint32_t) * (size_t)(m > 0 ? m : 1));
  uint32_t* c = malloc(sizeof(uint32_t) * (size_t)(m > 0 ? m : 1));

  or_exact_pairs(n, off, adj, m, eu, ev, a);
  const uint64_t exact_sum = sum32(a, m);
  const uint64_t tc = or_exact_tc_listing(n, off, adj);

  const uint32_t B = 320, W = B / 64;
  uint64_t* words = malloc(sizeof(uint64_t) * (size_t)n * W);
  uint32_t* pc = malloc(sizeof(uint32_t) * (size_t)n);
  or_bf_build(n, off, adj, B, 2, 7, words, pc);
  or_bf_counts(W, words, m, eu, ev, a, b);
  const uint64_t bf_and = sum32(a, m), bf_or = sum32(b, m), bf_pc = sum32(pc, n);

  const uint32_t k = 16;
  uint32_t* sig = malloc(sizeof(uint32_t) * (size_t)n * k);
  or_kh_build(n, off, adj, k, 9, sig);
  or_kh_counts(k, sig, m, eu, ev, a);
  const uint64_t kh = sum32(a, m);
  or_1h_build(n, off, adj, k, 11, sig);
  or_1h_counts(k, 11, sig, m, eu, ev, a, b, c);
  const uint64_t oh_su = sum32(a, m), oh_kp = sum32(b, m), oh_lit = sum32(c, m);

  const uint64_t ck = or_four_cliques(n, poff, padj, deg, NULL, 64, 1, 0);
  uint64_t* pwords = malloc(sizeof(uint64_t) * (size_t)n * 2);
  uint32_t* ppc = malloc(sizeof(uint32_t) * (size_t)n);
  or_bf_build(n, poff, padj, 128, 1, 5, pwords, ppc);
  const uint64_t ck_bf = or_four_cliques(n, poff, padj, deg, pwords, 128, 1, 5);
  uint64_t hist_and[129], hist_or[129], ck_sizes = 0, ck_and = 0, ck_or = 0;
  or_four_cliques_filters(n, poff, padj, pwords, 128, 1, 5, hist_and, hist_or, &ck_sizes);
  for (int t = 0; t <= 128; ++t) {
    ck_and += (uint64_t)t * hist_and[t];
    ck_or += (uint64_t)t * hist_or[t];
  }

  printf("%lld %llu %llu %llu %llu %llu %llu %llu %llu %llu %llu %llu %llu %llu %llu\n", (long long)m,
         (unsigned long long)tc,
         (unsigned long long)exact_sum, (unsigned long long)bf_and, (unsigned long long)bf_or,
         (unsigned long long)bf_pc, (unsigned long long)kh, (unsigned long long)oh_su, (unsigned long long)oh_kp,
         (unsigned long long)oh_lit, (unsigned long long)ck, (unsigned long long)ck_bf,
         (unsigned long long)ck_and, (unsigned long long)ck_or, (unsigned long long)ck_sizes);
  free(off); free(adj); free(poff); free(padj); free(deg); free(eu); free(ev); free(a); free(b); free(c);
  free(words); free(pc); free(sig); free(pwords); free(ppc);
  return 0;
}
