/*
 * ORACLE -- test infrastructure only.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  It shares no
 * code with the GPU decoder.
 *
 * Plain FP64 flooding sum-product decoding of a binary LDPC code (Sec. II-B,
 * Eqs. 4-8; flooding order of Algorithm 1), one codeword at a time, with
 * codewords split over threads by the block rule of Eq. 9 (read as
 * floor(l/N) + [x < l mod N] items for worker x).
 *
 * Conventions (the paper's sign mirrored, see the module docs):
 *   lambda_v = log P(c_v=0|y) / P(c_v=1|y); hard decision z_v = 1 iff L_v <= 0.
 *   Check rule (Eq. 5, denominator read as 1 - prod):
 *       E_cv = 2 atanh( prod_{v' in N(c), v' != v} tanh(M_v'c / 2) )
 *   Variable rule (Eq. 6):  M_vc = R_v + sum_{c' in N(v), c' != c} E_c'v,
 *       clamped to [-20, 20] (the paper is silent on saturation).
 *   Posterior (Eq. 7):      L_v = R_v + sum_{c in N(v)} E_cv.
 *   Early stop: the syndrome H z^T is tested on the channel decisions and after
 *   every iteration; the first zero syndrome ends the word (iterations used = t).
 * Products and sums run over the neighbours in ascending index order, written
 * out directly (no prefix/suffix or total-minus-self shortcuts).
 *
 * The unrolled weighted form multiplies every c->v message of iteration t by a
 * per-edge weight w[t][e] wherever it enters a variable-node sum:
 *       M^(t+1)_vc = clamp(R_v + sum_{c' != c} w^(t)_c'v E^(t)_c'v)
 *       L_v        = R_v + sum_c w^(T)_cv E^(T)_cv
 * with M^(1) = clamp(R).  All weights 1 gives the plain decoder without early stop.
 *
 * State in and out (for one-step checks and resumption): a decode may start from given
 * c->v messages E^(0) instead of zeros.  Then the iteration-0 posterior is Eq. 7 on that
 * state, L^(0) = R + sum_c E^(0)_cv, its decisions are tested first, and iteration 1
 * forms M^(1) from E^(0) by Eq. 6; with E^(0) = 0 this is the decode above.  The state
 * after the last iteration (E of iteration `iters`) can be returned.
 *
 * FP32-storage build (compiled with -DORACLE_STORE32): the same source, with every
 * value the decoder keeps between steps -- R, each c->v and v->c message, each
 * posterior -- rounded to FP32 where it is stored, while every formula is still
 * evaluated in FP64.  It is the decoder an FP32 implementation would be if each of
 * its stored values were correctly rounded, the reference point for how far FP32
 * storage alone moves posteriors along a decoding trajectory.  (A build with FP32
 * arithmetic throughout is not a usable reference: tanh(x / 2) rounds to 1 in FP32
 * for x above about 18, so the tanh rule meets atanh(1) = inf at the clamp.)
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define L_MAX 20.0

#ifdef ORACLE_STORE32
#define STORE(x) ((double)(float)(x))
#else
#define STORE(x) (x)
#endif

typedef struct {
  int32_t m, n;
  int64_t nnz;
  const int32_t *row_ptr, *col_idx; /* CSR of H: edge e of check c is e in [row_ptr[c], row_ptr[c+1]) */
  int64_t *var_ptr;                 /* edges of variable v: var_edges[var_ptr[v] .. var_ptr[v+1]) */
  int64_t *var_edges;               /* ascending edge id == ascending check index */
} graph_t;

static int graph_init(graph_t *g, int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx) {
  g->m = m;
  g->n = n;
  g->row_ptr = row_ptr;
  g->col_idx = col_idx;
  g->nnz = row_ptr[m];
  g->var_ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  g->var_edges = (int64_t *)malloc((size_t)(g->nnz > 0 ? g->nnz : 1) * sizeof(int64_t));
  if (!g->var_ptr || !g->var_edges) return -1;
  for (int64_t e = 0; e < g->nnz; e++) g->var_ptr[col_idx[e] + 1]++;
  for (int32_t v = 0; v < n; v++) g->var_ptr[v + 1] += g->var_ptr[v];
  int64_t *fill = (int64_t *)malloc((size_t)n * sizeof(int64_t) + 1);
  if (!fill) return -1;
  for (int32_t v = 0; v < n; v++) fill[v] = g->var_ptr[v];
  for (int64_t e = 0; e < g->nnz; e++) g->var_edges[fill[col_idx[e]]++] = e;
  free(fill);
  return 0;
}

static void graph_free(graph_t *g) {
  free(g->var_ptr);
  free(g->var_edges);
}

static double clamp_llr(double x) { return x > L_MAX ? L_MAX : (x < -L_MAX ? -L_MAX : x); }

/* z_v = 1 iff L_v <= 0 (a comparison, so +0 and -0 agree) */
static void hard_decide(const graph_t *g, const double *L, uint8_t *z) {
  for (int32_t v = 0; v < g->n; v++) z[v] = (L[v] <= 0.0) ? 1 : 0;
}

/* 1 iff H z^T = 0 over GF(2) (Eq. 1) */
static int syndrome_zero(const graph_t *g, const uint8_t *z) {
  for (int32_t c = 0; c < g->m; c++) {
    int par = 0;
    for (int64_t e = g->row_ptr[c]; e < g->row_ptr[c + 1]; e++) par ^= z[g->col_idx[e]];
    if (par) return 0;
  }
  return 1;
}

/* Eq. 6 with optional weights on the incoming c->v messages (w == NULL: weight 1). */
static void variable_messages(const graph_t *g, const double *R, const double *E, const double *w, double *M) {
  for (int32_t v = 0; v < g->n; v++) {
    for (int64_t i = g->var_ptr[v]; i < g->var_ptr[v + 1]; i++) {
      int64_t e = g->var_edges[i];
      double s = R[v];
      for (int64_t j = g->var_ptr[v]; j < g->var_ptr[v + 1]; j++) {
        int64_t f = g->var_edges[j];
        if (f == e) continue;
        s += w ? w[f] * E[f] : E[f];
      }
      M[e] = STORE(clamp_llr(s));
    }
  }
}

/* Eq. 5 (tanh rule), every check, every edge */
static void check_messages(const graph_t *g, const double *M, double *E) {
  for (int32_t c = 0; c < g->m; c++) {
    for (int64_t e = g->row_ptr[c]; e < g->row_ptr[c + 1]; e++) {
      double p = 1.0;
      for (int64_t f = g->row_ptr[c]; f < g->row_ptr[c + 1]; f++) {
        if (f == e) continue;
        p *= tanh(M[f] / 2.0);
      }
      E[e] = STORE(2.0 * atanh(p));
    }
  }
}

/* Eq. 7 */
static void posterior(const graph_t *g, const double *R, const double *E, const double *w, double *L) {
  for (int32_t v = 0; v < g->n; v++) {
    double s = R[v];
    for (int64_t i = g->var_ptr[v]; i < g->var_ptr[v + 1]; i++) {
      int64_t e = g->var_edges[i];
      s += w ? w[e] * E[e] : E[e];
    }
    L[v] = STORE(s);
  }
}

typedef struct {
  double *E, *M, *R;
  uint8_t *z;
} scratch_t;

static int scratch_alloc(scratch_t *s, const graph_t *g) {
  size_t ne = (size_t)(g->nnz > 0 ? g->nnz : 1);
  s->E = (double *)malloc(ne * sizeof(double));
  s->M = (double *)malloc(ne * sizeof(double));
  s->R = (double *)malloc(((size_t)g->n + 1) * sizeof(double));
  s->z = (uint8_t *)malloc((size_t)g->n + 1);
  return (s->E && s->M && s->R && s->z) ? 0 : -1;
}

static void scratch_free(scratch_t *s) {
  free(s->E);
  free(s->M);
  free(s->R);
  free(s->z);
}

/* One codeword of the plain decoder.  L receives the posterior.  E0 (nullable) is the
 * starting c->v state [nnz]; Eout (nullable) receives the state of the last iteration. */
static void decode_word(const graph_t *g, const double *Rin, int32_t T, int32_t early_stop, scratch_t *s,
                        const double *E0, double *Eout, double *L, uint8_t *hard, int32_t *iters, uint8_t *conv) {
  double *R = s->R;
  for (int32_t v = 0; v < g->n; v++) R[v] = STORE(Rin[v]);
  if (E0) {
    for (int64_t e = 0; e < g->nnz; e++) s->E[e] = STORE(E0[e]);
    posterior(g, R, s->E, NULL, L);
  } else {
    for (int64_t e = 0; e < g->nnz; e++) s->E[e] = 0.0;
    for (int32_t v = 0; v < g->n; v++) L[v] = R[v];
  }
  hard_decide(g, L, s->z);
  int32_t t = 0;
  int ok = syndrome_zero(g, s->z);
  if (!(early_stop && ok)) {
    for (t = 1; t <= T; t++) {
      variable_messages(g, R, s->E, NULL, s->M);
      check_messages(g, s->M, s->E);
      posterior(g, R, s->E, NULL, L);
      hard_decide(g, L, s->z);
      ok = syndrome_zero(g, s->z);
      if (early_stop && ok) break;
    }
    if (t > T) t = T;
  }
  memcpy(hard, s->z, (size_t)g->n);
  if (Eout) memcpy(Eout, s->E, (size_t)g->nnz * sizeof(double));
  *iters = t;
  *conv = (uint8_t)ok;
}

/* One codeword of the unrolled weighted form: T iterations, no early stop. */
static void unrolled_word(const graph_t *g, const double *R, int32_t T, const double *w, scratch_t *s, double *L) {
  for (int64_t e = 0; e < g->nnz; e++) s->E[e] = 0.0;
  const double *wprev = NULL;
  for (int32_t t = 1; t <= T; t++) {
    if (t == 1) {
      for (int32_t v = 0; v < g->n; v++)
        for (int64_t i = g->var_ptr[v]; i < g->var_ptr[v + 1]; i++) s->M[g->var_edges[i]] = clamp_llr(R[v]);
    } else {
      variable_messages(g, R, s->E, wprev, s->M);
    }
    check_messages(g, s->M, s->E);
    wprev = w + (size_t)(t - 1) * (size_t)g->nnz;
  }
  if (T == 0) {
    for (int32_t v = 0; v < g->n; v++) L[v] = R[v];
    return;
  }
  posterior(g, R, s->E, wprev, L);
}

typedef struct {
  const graph_t *g;
  const double *llr;
  int64_t b0, b1;
  int32_t T, early_stop;
  const double *w; /* unrolled form when non-NULL or when mode == 1 */
  const double *E0; /* starting c->v state [B][nnz] (plain form, nullable) */
  double *Eout;     /* final c->v state [B][nnz] (plain form, nullable) */
  int mode;        /* 0 plain, 1 unrolled */
  uint8_t *hard;
  double *post;
  int32_t *iters;
  uint8_t *conv;
  int status;
} job_t;

static void *worker(void *arg) {
  job_t *j = (job_t *)arg;
  scratch_t s;
  if (scratch_alloc(&s, j->g)) {
    j->status = -1;
    scratch_free(&s);
    return NULL;
  }
  const int32_t n = j->g->n;
  for (int64_t b = j->b0; b < j->b1; b++) {
    const double *R = j->llr + (size_t)b * n;
    const size_t eo = (size_t)b * (size_t)j->g->nnz;
    if (j->mode == 0)
      decode_word(j->g, R, j->T, j->early_stop, &s, j->E0 ? j->E0 + eo : NULL, j->Eout ? j->Eout + eo : NULL,
                  j->post + (size_t)b * n, j->hard + (size_t)b * n, j->iters + b, j->conv + b);
    else
      unrolled_word(j->g, R, j->T, j->w, &s, j->post + (size_t)b * n);
  }
  scratch_free(&s);
  j->status = 0;
  return NULL;
}

static int run_jobs(job_t *proto, int64_t B, int32_t nthreads) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > B) nthreads = (int32_t)(B > 0 ? B : 1);
  job_t *jobs = (job_t *)calloc((size_t)nthreads, sizeof(job_t));
  pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
  char *created = (char *)calloc((size_t)nthreads, 1); /* read and written by this thread only */
  if (!jobs || !th || !created) {
    free(jobs);
    free(th);
    free(created);
    return -1;
  }
  /* Eq. 9 block split: worker x gets floor(B/N) + [x < B mod N] consecutive words */
  int64_t q = B / nthreads, r = B % nthreads, start = 0;
  for (int32_t x = 0; x < nthreads; x++) {
    jobs[x] = *proto;
    int64_t cnt = q + (x < r ? 1 : 0);
    jobs[x].b0 = start;
    jobs[x].b1 = start + cnt;
    start += cnt;
  }
  int rc = 0;
  for (int32_t x = 1; x < nthreads; x++) {
    created[x] = pthread_create(&th[x], NULL, worker, &jobs[x]) == 0;
    if (!created[x]) worker(&jobs[x]); /* no thread: this one does the share */
  }
  worker(&jobs[0]);
  for (int32_t x = 1; x < nthreads; x++)
    if (created[x]) pthread_join(th[x], NULL);
  for (int32_t x = 0; x < nthreads; x++) /* every worker has finished: statuses are final */
    if (jobs[x].status == -1) rc = -1;
  free(jobs);
  free(th);
  free(created);
  return rc;
}

/* Plain decoder: llr [B][n] FP64 -> hard [B][n] (0/1), post [B][n], iters [B], conv [B].
 * init_cv [B][nnz] (nullable): starting c->v messages, CSR edge order; final_cv [B][nnz]
 * (nullable) receives the c->v messages of each word's last iteration. */
int oracle_decode_ex(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *llr,
                     int64_t B, int32_t max_iters, int32_t early_stop, int32_t nthreads, const double *init_cv,
                     double *final_cv, uint8_t *hard, double *post, int32_t *iters, uint8_t *conv) {
  graph_t g;
  if (m <= 0 || n <= 0 || max_iters < 0 || B < 0) return -3;
  if (graph_init(&g, m, n, row_ptr, col_idx)) {
    graph_free(&g);
    return -1;
  }
  job_t proto;
  memset(&proto, 0, sizeof(proto));
  proto.g = &g;
  proto.llr = llr;
  proto.T = max_iters;
  proto.early_stop = early_stop;
  proto.mode = 0;
  proto.E0 = init_cv;
  proto.Eout = final_cv;
  proto.hard = hard;
  proto.post = post;
  proto.iters = iters;
  proto.conv = conv;
  int rc = B > 0 ? run_jobs(&proto, B, nthreads) : 0;
  graph_free(&g);
  return rc;
}

int oracle_decode(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *llr,
                  int64_t B, int32_t max_iters, int32_t early_stop, int32_t nthreads, uint8_t *hard, double *post,
                  int32_t *iters, uint8_t *conv) {
  return oracle_decode_ex(m, n, row_ptr, col_idx, llr, B, max_iters, early_stop, nthreads, NULL, NULL, hard, post,
                          iters, conv);
}

/* Unrolled weighted form: w [T][nnz] FP64 -> post [B][n]. */
int oracle_unrolled(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *llr,
                    int64_t B, int32_t T, const double *w, int32_t nthreads, double *post) {
  graph_t g;
  if (m <= 0 || n <= 0 || T < 0 || B < 0) return -3;
  if (graph_init(&g, m, n, row_ptr, col_idx)) {
    graph_free(&g);
    return -1;
  }
  job_t proto;
  memset(&proto, 0, sizeof(proto));
  proto.g = &g;
  proto.llr = llr;
  proto.T = T;
  proto.w = w;
  proto.mode = 1;
  proto.post = post;
  int rc = B > 0 ? run_jobs(&proto, B, nthreads) : 0;
  graph_free(&g);
  return rc;
}

/* H z^T = 0 test for words [B][n]: ok[b] = 1 iff every parity check of word b holds. */
int oracle_syndrome_ok(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const uint8_t *words,
                       int64_t B, uint8_t *ok) {
  graph_t g;
  g.m = m;
  g.n = n;
  g.row_ptr = row_ptr;
  g.col_idx = col_idx;
  for (int64_t b = 0; b < B; b++) ok[b] = (uint8_t)syndrome_zero(&g, words + (size_t)b * n);
  return 0;
}
