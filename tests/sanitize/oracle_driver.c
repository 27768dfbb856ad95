/* Runs every oracle routine on small graphs under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built by tests/test_sanitize.py with
 * -fsanitize=address,undefined); checks closed forms and that the routines
 * agree, and exits non-zero on any mismatch.  Test infrastructure. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t oracle_normalise(const int32_t *src, const int32_t *dst, int64_t n_pairs, int32_t n,
                         int32_t one_based, int32_t *u_out, int32_t *v_out);
int64_t oracle_triangle_count(int32_t n, int64_t m, const int32_t *u, const int32_t *v);
int64_t oracle_triangle_count_threads(int32_t n, int64_t m, const int32_t *u, const int32_t *v,
                                      int32_t nthreads);
int oracle_support(int32_t n, int64_t m, const int32_t *u, const int32_t *v, int32_t *s);
int oracle_support_listing(int32_t n, int64_t m, const int32_t *u, const int32_t *v, int32_t *s);
int32_t oracle_ktruss_bulk(int32_t n, int64_t m, const int32_t *u, const int32_t *v, int32_t k,
                           uint8_t *in_out);
int32_t oracle_ktruss_peel(int32_t n, int64_t m, const int32_t *u, const int32_t *v, int32_t k,
                           uint8_t *in_out);
int32_t oracle_ktruss_search(int32_t n, int64_t m, const int32_t *u, const int32_t *v, int32_t k,
                             uint8_t *in_out);
int oracle_truss_decomposition(int32_t n, int64_t m, const int32_t *u, const int32_t *v,
                               int32_t method, int32_t *tau, int32_t *kmax);

static int failures = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      ++failures;                                                  \
    }                                                              \
  } while (0)

static uint64_t lcg = 88172645463325252ull;
static uint32_t rnd(void) {
  lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
  return (uint32_t)(lcg >> 33);
}

/* every routine on one raw pair list; T_want < 0: no closed form */
static void run(const char *name, int32_t n, const int32_t *src, const int32_t *dst, int64_t P,
                int64_t T_want, int32_t kmax_want) {
  int32_t *u = malloc(sizeof(int32_t) * (size_t)(P + 1));
  int32_t *v = malloc(sizeof(int32_t) * (size_t)(P + 1));
  const int64_t m = oracle_normalise(src, dst, P, n, 0, u, v);
  CHECK(m >= 0);
  const int64_t T = oracle_triangle_count(n, m, u, v);
  if (T_want >= 0) CHECK(T == T_want);
  for (int32_t th = 1; th <= 4; th += 3) CHECK(oracle_triangle_count_threads(n, m, u, v, th) == T);
  int32_t *s1 = calloc((size_t)m + 1, sizeof(int32_t)), *s2 = calloc((size_t)m + 1, sizeof(int32_t));
  CHECK(oracle_support(n, m, u, v, s1) == 0);
  CHECK(oracle_support_listing(n, m, u, v, s2) == 0);
  int64_t sum = 0;
  for (int64_t e = 0; e < m; ++e) { CHECK(s1[e] == s2[e]); sum += s1[e]; }
  CHECK(sum == 3 * T);
  int32_t *tau[3];
  int32_t km[3];
  for (int meth = 0; meth < 3; ++meth) {
    tau[meth] = calloc((size_t)m + 1, sizeof(int32_t));
    CHECK(oracle_truss_decomposition(n, m, u, v, meth, tau[meth], &km[meth]) == 0);
  }
  if (kmax_want >= 0) CHECK(km[0] == kmax_want);
  CHECK(km[0] == km[1] && km[0] == km[2]);
  for (int64_t e = 0; e < m; ++e) CHECK(tau[0][e] == tau[1][e] && tau[0][e] == tau[2][e]);
  uint8_t *mk[3];
  for (int k = 2; k <= km[0] + 1; ++k) {
    for (int i = 0; i < 3; ++i) {
      mk[i] = malloc((size_t)m + 1);
      memset(mk[i], 1, (size_t)m + 1);
    }
    CHECK(oracle_ktruss_bulk(n, m, u, v, k, mk[0]) >= 0);
    CHECK(oracle_ktruss_peel(n, m, u, v, k, mk[1]) == 0);
    CHECK(oracle_ktruss_search(n, m, u, v, k, mk[2]) == 0);
    for (int64_t e = 0; e < m; ++e) {
      CHECK(mk[0][e] == mk[1][e] && mk[0][e] == mk[2][e]);
      CHECK(mk[0][e] == (tau[0][e] >= k));
    }
    for (int i = 0; i < 3; ++i) free(mk[i]);
  }
  for (int meth = 0; meth < 3; ++meth) free(tau[meth]);
  free(s1); free(s2); free(u); free(v);
  fprintf(stderr, "%s: m=%lld T=%lld kmax=%d\n", name, (long long)m, (long long)T, km[0]);
}

int main(void) {
  /* complete graphs K_n: C(n,3) triangles, kmax n; pairs in both directions,
     with a self-loop and a repeat */
  for (int32_t nk = 1; nk <= 24; nk += 7) {
    const int64_t P = (int64_t)nk * nk + 2;
    int32_t *s = malloc(sizeof(int32_t) * P), *d = malloc(sizeof(int32_t) * P);
    int64_t q = 0;
    for (int32_t a = 0; a < nk; ++a)
      for (int32_t b = 0; b < nk; ++b) { s[q] = a; d[q] = b; ++q; }
    s[q] = 0; d[q] = 0; ++q;
    s[q] = nk > 1 ? 1 : 0; d[q] = 0; ++q;
    run("complete", nk, s, d, q, (int64_t)nk * (nk - 1) * (nk - 2) / 6, nk >= 2 ? nk : 0);
    free(s); free(d);
  }
  /* king graph M x M: 4 (M-1)^2 triangles, kmax 4 */
  {
    const int32_t M = 9, n = M * M;
    int32_t s[4 * 81], d[4 * 81];
    int64_t q = 0;
    for (int32_t r = 0; r < M; ++r)
      for (int32_t c = 0; c < M; ++c) {
        const int32_t x = r * M + c;
        if (c + 1 < M) { s[q] = x; d[q++] = x + 1; }
        if (r + 1 < M) { s[q] = x; d[q++] = x + M; }
        if (r + 1 < M && c + 1 < M) { s[q] = x; d[q++] = x + M + 1; }
        if (r + 1 < M && c > 0) { s[q] = x; d[q++] = x + M - 1; }
      }
    run("king", n, s, d, q, 4LL * (M - 1) * (M - 1), 4);
  }
  /* random graphs of several densities */
  for (int trial = 0; trial < 12; ++trial) {
    const int32_t n = 8 + (int32_t)(rnd() % 120);
    const int64_t P = 1 + rnd() % (uint32_t)(n * 6);
    int32_t *s = malloc(sizeof(int32_t) * P), *d = malloc(sizeof(int32_t) * P);
    for (int64_t i = 0; i < P; ++i) { s[i] = (int32_t)(rnd() % (uint32_t)n); d[i] = (int32_t)(rnd() % (uint32_t)n); }
    run("random", n, s, d, P, -1, -1);
    free(s); free(d);
  }
  /* empty graph and a vertex id out of range */
  {
    int32_t s[1] = {0}, d[1] = {0};
    run("empty", 4, s, d, 0, 0, 0);
    int32_t u[2], v[2];
    int32_t bad_s[1] = {3}, bad_d[1] = {7};
    CHECK(oracle_normalise(bad_s, bad_d, 1, 5, 0, u, v) == -1);
  }
  if (failures) fprintf(stderr, "%d checks failed\n", failures);
  return failures ? 1 : 0;
}
