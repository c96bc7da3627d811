// Plain flooding sum-product decoder: one workgroup per 64-word tile.
//
// The batch is cut into tiles of 64 words (Sec. III-C's batch split: every
// worker decodes whole words).  A workgroup of W wavefronts owns one tile for
// the whole decode; its waves split the checks and the variables of the graph
// in the interleaved way of Algorithm 1 (check c and variable v go to wave
// c mod W and v mod W), with a workgroup barrier where Algorithm 1 exchanges
// messages.  Messages of the tile live in HBM as [edge][64] FP32, the posterior
// and the channel LLRs as [variable][64].
//
// Per iteration (flooding, Algorithm 1):
//   check phase     every check: syndrome bit of the current decisions, new E (Eq. 5)
//   decide          lanes whose decisions satisfy H z^T = 0 (Eq. 1), or that reached
//                   max_iters, stop; their posterior stays frozen
//   variable phase  every variable: L = R + sum E (Eq. 7) for the lanes still running
// The check phase of the step that detects convergence also produces messages
// for that lane, which are discarded (its stores are kept, its L is not updated).
#include "internal.h"
#include "spa_core.h"

namespace ldpc {

// [B][n] channel LLRs -> tile layout [n][64] of R and L, through 64 x 64 LDS blocks.
__device__ __forceinline__ void ingest_tile(const float *__restrict__ llr32, const double *__restrict__ llr64, int n,
                                            int cw0, int nvalid, float *__restrict__ Rt, float *__restrict__ Lt,
                                            float (*stage)[TW + 1], int wave, int W, int lane) {
  for (int v0 = 0; v0 < n; v0 += TW) {
    for (int r = wave; r < TW; r += W) {
      float x = 0.0f;
      const int v = v0 + lane;
      if (r < nvalid && v < n) {
        const size_t off = (size_t)(cw0 + r) * (size_t)n + (size_t)v;
        x = llr64 ? (float)llr64[off] : llr32[off];
      }
      stage[r][lane] = x;
    }
    __syncthreads();
    for (int q = wave; q < TW && v0 + q < n; q += W) {
      const float x = stage[lane][q];
      Rt[(v0 + q) * TW + lane] = x;
      Lt[(v0 + q) * TW + lane] = x;
    }
    __syncthreads();
  }
}

// Tile layout [n][64] of L -> posterior and hard decisions [B][n].
__device__ __forceinline__ void egress_tile(const float *__restrict__ Lt, int n, int cw0, int nvalid,
                                            float *__restrict__ post, uint8_t *__restrict__ hard,
                                            float (*stage)[TW + 1], int wave, int W, int lane) {
  for (int v0 = 0; v0 < n; v0 += TW) {
    for (int q = wave; q < TW && v0 + q < n; q += W) stage[q][lane] = Lt[(v0 + q) * TW + lane];
    __syncthreads();
    for (int r = wave; r < nvalid; r += W) {
      const int v = v0 + lane;
      if (v < n) {
        const float x = stage[lane][r];
        const size_t off = (size_t)(cw0 + r) * (size_t)n + (size_t)v;
        post[off] = x;
        hard[off] = x <= 0.0f ? 1 : 0;
      }
    }
    __syncthreads();
  }
}

template <int DC, int DV>
__global__ void __launch_bounds__(1024)
    plain_decode_kernel(GraphDev g, const float *__restrict__ llr32, const double *__restrict__ llr64, int B,
                        int max_iters, int early_stop, float *__restrict__ wsE, float *__restrict__ wsL,
                        float *__restrict__ wsR, uint8_t *__restrict__ hard, float *__restrict__ post,
                        int32_t *__restrict__ iters) {
  __shared__ float stage[TW][TW + 1];
  __shared__ unsigned long long unsat_w[16];
  const int lane = lane_id();
  const int wave = wave_id();
  const int W = blockDim.x >> 6;
  const int tile = blockIdx.x;
  const int cw0 = tile * TW;
  const int nvalid = min(TW, B - cw0);
  float *Et = wsE + (size_t)tile * (size_t)g.nnz * TW;
  float *Lt = wsL + (size_t)tile * (size_t)g.n * TW;
  float *Rt = wsR + (size_t)tile * (size_t)g.n * TW;

  ingest_tile(llr32, llr64, g.n, cw0, nvalid, Rt, Lt, stage, wave, W, lane);

  bool active = lane < nvalid;
  int my_iters = 0;
  for (int it = 0;; ++it) {
    // check phase
    int unsat = 0;
    const bool use_old = it > 0;
    for (int c = wave; c < g.m; c += W) {
      int e0, dc;
      if (DC > 0) {
        e0 = c * DC;
        dc = DC;
      } else {
        e0 = g.row_ptr[c];
        dc = g.row_ptr[c + 1] - e0;
      }
      unsat |= check_update<DC>(Lt, Et, g.col_idx, e0, dc, lane, use_old, active);
    }
    const unsigned long long b = __ballot(unsat);
    if (lane == 0) unsat_w[wave] = b;
    __syncthreads();
    unsigned long long um = 0;
    for (int w = 0; w < W; ++w) um |= unsat_w[w];
    const bool lane_unsat = (um >> lane) & 1ull;
    if (active && ((early_stop && !lane_unsat) || it == max_iters)) {
      active = false;
      my_iters = it;
    }
    if (__ballot(active) == 0ull) break;  // same value in every wave of the workgroup
    // variable phase
    for (int v = wave; v < g.n; v += W) {
      int p0, dv;
      if (DV > 0) {
        p0 = v * DV;
        dv = DV;
      } else {
        p0 = g.var_ptr[v];
        dv = g.var_ptr[v + 1] - p0;
      }
      const float s = var_sum<DV>(Rt, Et, g.var_edges, p0, dv, v, lane);
      if (active) Lt[v * TW + lane] = s;
    }
    __syncthreads();
  }

  egress_tile(Lt, g.n, cw0, nvalid, post, hard, stage, wave, W, lane);
  if (wave == 0 && lane < nvalid) iters[cw0 + lane] = my_iters;
}

}  // namespace ldpc

using namespace ldpc;

size_t plain_workspace_bytes(const ldpc_graph_s *g, int32_t batch) {
  const size_t tiles = ((size_t)batch + TW - 1) / TW;
  return align256(tiles * (size_t)g->nnz * TW * sizeof(float)) +
         2 * align256(tiles * (size_t)g->n * TW * sizeof(float));
}

namespace {

using PlainKernel = void (*)(GraphDev, const float *, const double *, int, int, int, float *, float *, float *,
                             uint8_t *, float *, int32_t *);

PlainKernel pick_plain(const ldpc_graph_s *g, const GraphDev &d) {
#define LDPC_CASE(C, V) \
  if (d.dc == C && d.dv == V) return plain_decode_kernel<C, V>;
  LDPC_CASE(6, 3)
  LDPC_CASE(4, 3)
  LDPC_CASE(12, 3)
  LDPC_CASE(15, 3)
  LDPC_CASE(12, 6)
  LDPC_CASE(12, 9)
#undef LDPC_CASE
  if (g->dc_max <= 8) return plain_decode_kernel<-8, -LDPC_MAX_VAR_DEGREE>;
  if (g->dc_max <= 16) return plain_decode_kernel<-16, -LDPC_MAX_VAR_DEGREE>;
  if (g->dc_max <= 24) return plain_decode_kernel<-24, -LDPC_MAX_VAR_DEGREE>;
  return plain_decode_kernel<-LDPC_MAX_CHECK_DEGREE, -LDPC_MAX_VAR_DEGREE>;
}

}  // namespace

ldpc_status launch_plain_decode(const ldpc_graph_s *g, const void *llr, bool llr_f64, int32_t batch,
                                int32_t max_iters, int32_t early_stop, uint8_t *hard, float *post, int32_t *iters,
                                void *ws, size_t ws_bytes, int32_t waves, hipStream_t stream) {
  (void)ws_bytes;
  GraphDev d = graph_dev(g);
  const size_t tiles = ((size_t)batch + TW - 1) / TW;
  char *p = (char *)ws;
  float *wsE = (float *)p;
  p += align256(tiles * (size_t)g->nnz * TW * sizeof(float));
  float *wsL = (float *)p;
  p += align256(tiles * (size_t)g->n * TW * sizeof(float));
  float *wsR = (float *)p;
  PlainKernel k = pick_plain(g, d);
  const float *l32 = llr_f64 ? nullptr : (const float *)llr;
  const double *l64 = llr_f64 ? (const double *)llr : nullptr;
  hipLaunchKernelGGL(k, dim3((unsigned)tiles), dim3(64 * waves), 0, stream, d, l32, l64, (int)batch, (int)max_iters,
                     (int)(early_stop != 0), wsE, wsL, wsR, hard, post, iters);
  LDPC_HIP_CHECK(hipGetLastError());
  return LDPC_OK;
}
