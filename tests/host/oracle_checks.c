/* The FP64 oracle (oracle/spa.c) driven under the address and undefined-behaviour
 * sanitizers by tests/test_host_sanitizers.py: every entry point on seeded random codes,
 * with several threads, edge-case sizes (one word, zero iterations, variables of degree 0)
 * and the state-in/state-out decode.  Checks return codes and two exact properties:
 * noiseless words stop at iteration 0, and resuming from an exported state equals a
 * continuous decode. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_decode(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *llr, int64_t B,
                  int32_t max_iters, int32_t early_stop, int32_t nthreads, uint8_t *hard, double *post, int32_t *iters,
                  uint8_t *conv);
int oracle_decode_ex(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *llr,
                     int64_t B, int32_t max_iters, int32_t early_stop, int32_t nthreads, const double *init_cv,
                     double *final_cv, uint8_t *hard, double *post, int32_t *iters, uint8_t *conv);
int oracle_unrolled(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *llr,
                    int64_t B, int32_t T, const double *w, int32_t nthreads, double *post);
int oracle_syndrome_ok(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const uint8_t *words,
                       int64_t B, uint8_t *ok);

static uint64_t st = 88172645463325252ull;
static uint64_t rnd(void) {
  st ^= st << 13;
  st ^= st >> 7;
  st ^= st << 17;
  return st;
}
static double unif(void) { return (double)(rnd() >> 11) * (1.0 / 9007199254740992.0); }

static int failures = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);   \
      failures++;                                                       \
    }                                                                   \
  } while (0)

int main(void) {
  for (int trial = 0; trial < 12; trial++) {
    const int n = 8 + (int)(rnd() % 60), m = 3 + (int)(rnd() % (unsigned)(n / 2));
    int32_t *ptr = malloc(sizeof(int32_t) * (m + 1));
    int32_t *idx = malloc(sizeof(int32_t) * m * n);
    int nnz = 0;
    ptr[0] = 0;
    for (int c = 0; c < m; c++) { /* degree 2..min(9, n); some variables may end with degree 0 */
      const int d = 2 + (int)(rnd() % 8);
      int picked = 0;
      for (int v = 0; v < n && picked < d; v++)
        if (rnd() % (unsigned)(n - v) < (unsigned)(d - picked)) {
          idx[nnz++] = v;
          picked++;
        }
      ptr[c + 1] = nnz;
    }
    const int B = 1 + (int)(rnd() % 9), T = (int)(rnd() % 12);
    double *llr = malloc(sizeof(double) * B * n), *post = malloc(sizeof(double) * B * n);
    double *post2 = malloc(sizeof(double) * B * n), *E = malloc(sizeof(double) * B * nnz);
    double *E2 = malloc(sizeof(double) * B * nnz), *w = malloc(sizeof(double) * (T + 1) * nnz);
    uint8_t *hard = malloc(B * n), *conv = malloc(B), *ok = malloc(B), *zero = calloc(B * n, 1);
    int32_t *it = malloc(sizeof(int32_t) * B), *it2 = malloc(sizeof(int32_t) * B);
    for (int i = 0; i < B * n; i++) llr[i] = 4.0 * unif() - 1.0;
    for (int i = 0; i < (T + 1) * nnz; i++) w[i] = 0.8 + 0.4 * unif();
    CHECK(oracle_decode(m, n, ptr, idx, llr, B, T, 1, 3, hard, post, it, conv) == 0);
    CHECK(oracle_syndrome_ok(m, n, ptr, idx, hard, B, ok) == 0);
    for (int b = 0; b < B; b++) CHECK(it[b] >= 0 && it[b] <= T && (int)ok[b] == (int)conv[b]);
    CHECK(oracle_unrolled(m, n, ptr, idx, llr, B, T, T ? w : NULL, 2, post) == 0);
    /* resume: t iterations, export, then the rest from the state = continuous decode */
    const int t1 = T / 2;
    CHECK(oracle_decode_ex(m, n, ptr, idx, llr, B, t1, 0, 2, NULL, E, hard, post, it, conv) == 0);
    CHECK(oracle_decode_ex(m, n, ptr, idx, llr, B, T - t1, 0, 2, E, E2, hard, post2, it2, conv) == 0);
    CHECK(oracle_decode_ex(m, n, ptr, idx, llr, B, T, 0, 4, NULL, E, hard, post, it, conv) == 0);
    CHECK(memcmp(post, post2, sizeof(double) * B * n) == 0);
    CHECK(T == 0 || memcmp(E, E2, sizeof(double) * B * nnz) == 0);
    /* noiseless all-zero word: stops at iteration 0 */
    for (int i = 0; i < B * n; i++) llr[i] = 3.0;
    CHECK(oracle_decode(m, n, ptr, idx, llr, B, T, 1, 2, hard, post, it, conv) == 0);
    for (int b = 0; b < B; b++) CHECK(it[b] == 0 && conv[b] == 1);
    CHECK(oracle_syndrome_ok(m, n, ptr, idx, zero, B, ok) == 0);
    for (int b = 0; b < B; b++) CHECK(ok[b] == 1);
    free(ptr); free(idx); free(llr); free(post); free(post2); free(E); free(E2); free(w);
    free(hard); free(conv); free(ok); free(zero); free(it); free(it2);
  }
  { /* refused sizes */
    int32_t ptr[2] = {0, 2}, idx[2] = {0, 1};
    double llr[2] = {1, 1}, post[2];
    uint8_t hard[2], conv[1];
    int32_t it[1];
    CHECK(oracle_decode(0, 2, ptr, idx, llr, 1, 5, 1, 1, hard, post, it, conv) != 0);
    CHECK(oracle_decode(1, 2, ptr, idx, llr, 1, -1, 1, 1, hard, post, it, conv) != 0);
    CHECK(oracle_decode(1, 2, ptr, idx, llr, 0, 5, 1, 1, hard, post, it, conv) == 0);
  }
  if (failures) {
    fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  printf("oracle checks ok\n");
  return 0;
}
