// Plain flooding sum-product decoder: one workgroup per 64-word tile.
//
// The batch is cut into tiles of 64 words (the batch split of Sec. III-C: every
// worker decodes whole words).  A workgroup of W wavefronts owns one tile for the
// whole decode; its waves split the checks and the variables of the graph in the
// interleaved way of Algorithm 1 (check c and variable v go to wave c mod W and
// v mod W), with a workgroup barrier where Algorithm 1 exchanges messages.
//
// HBM state of a tile (all FP32 [index][64] unless noted):
//   M  [nnz]  v->c messages (Eq. 6, clamped)       R [n]  channel LLRs (Eq. 4)
//   E0/E1 [nnz] c->v messages of even / odd iterations (Eq. 5)
//   Z  [n] u64 decision masks, bit l = z_v of lane l's word (Eq. 8)
// Iteration t+1 (flooding, Algorithm 1):
//   check phase     every check: syndrome bit of z^(t), E^(t+1) from M^(t+1) into E[(t+1)&1]
//   decide          a lane whose z^(t) satisfies H z^T = 0 (Eq. 1), or with t = max_iters,
//                   stops at t; from then on nothing of it is written, so its E^(t) stays
//                   in E[t&1]
//   variable phase  every variable: L^(t+1) (Eq. 7) -> Z, and M^(t+2) (Eq. 6) for running lanes
// The egress recomputes each word's final posterior from its own E buffer with the
// same summation as the variable phase, so it equals the L whose decisions stopped it.
#include "internal.h"
#include "spa_core.h"

namespace ldpc {

struct TileState {
  float *E0, *E1, *M, *R;
  unsigned long long *Z;
};

__device__ __forceinline__ TileState tile_state(float *wsE0, float *wsE1, float *wsM, float *wsR,
                                                unsigned long long *wsZ, const GraphDev &g, int tile) {
  TileState s;
  const size_t eoff = (size_t)tile * (size_t)g.nnz * TW;
  const size_t voff = (size_t)tile * (size_t)g.n * TW;
  s.E0 = wsE0 + eoff;
  s.E1 = wsE1 + eoff;
  s.M = wsM + eoff;
  s.R = wsR + voff;
  s.Z = wsZ + (size_t)tile * (size_t)g.n;
  return s;
}

template <int DV>
__device__ __forceinline__ void var_range(const GraphDev &g, int v, int &p0, int &dv) {
  if (DV > 0) {
    p0 = v * DV;
    dv = DV;
  } else {
    p0 = g.var_ptr[v];
    dv = g.var_ptr[v + 1] - p0;
  }
}

template <int DC>
__device__ __forceinline__ void check_range(const GraphDev &g, int c, int &e0, int &dc) {
  if (DC > 0) {
    e0 = c * DC;
    dc = DC;
  } else {
    e0 = g.row_ptr[c];
    dc = g.row_ptr[c + 1] - e0;
  }
}

// [B][n] channel LLRs -> R of the tile (through 64 x 64 LDS blocks), the first
// v->c messages M = clamp(R) on every edge, and the channel decisions Z.
template <int DV>
__device__ __forceinline__ void ingest_tile(const GraphDev &g, const float *__restrict__ llr32,
                                            const double *__restrict__ llr64, int cw0, int nvalid, TileState st,
                                            float (*stage)[TW + 1], int wave, int W, int lane) {
  const int n = g.n;
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
      const int v = v0 + q;
      const float x = stage[lane][q];
      st.R[v * TW + lane] = x;
      const unsigned long long z = __ballot(x <= 0.0f);
      if (lane == 0) st.Z[v] = z;
      int p0, dv;
      var_range<DV>(g, v, p0, dv);
      const float mx = clamp_msg(x);
      for (int j = 0; j < dv; ++j) st.M[g.var_edges[p0 + j] * TW + lane] = mx;
    }
    __syncthreads();
  }
}

// Final posterior of each lane's word from its own E buffer -> post and hard [B][n].
template <int DV>
__device__ __forceinline__ void egress_tile(const GraphDev &g, TileState st, int my_iters, int cw0, int nvalid,
                                            float *__restrict__ post, uint8_t *__restrict__ hard,
                                            float (*stage)[TW + 1], int wave, int W, int lane) {
  constexpr int DMAX = DV > 0 ? DV : -DV;
  const int n = g.n;
  const float *Eb = (my_iters & 1) ? st.E1 : st.E0;
  for (int v0 = 0; v0 < n; v0 += TW) {
    for (int q = wave; q < TW && v0 + q < n; q += W) {
      const int v = v0 + q;
      int p0, dv;
      var_range<DV>(g, v, p0, dv);
      float ev[DMAX], pre[DMAX];
      int eid[DMAX];
      const float r = st.R[v * TW + lane];
      const float L = var_posterior<DV>(r, Eb, g.var_edges, p0, dv, lane, ev, pre, eid);
      stage[q][lane] = my_iters > 0 ? L : r;
    }
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
                        int max_iters, int early_stop, float *wsE0, float *wsE1, float *wsM, float *wsR,
                        unsigned long long *wsZ, uint8_t *__restrict__ hard, float *__restrict__ post,
                        int32_t *__restrict__ iters) {
  __shared__ float stage[TW][TW + 1];
  __shared__ unsigned long long unsat_w[16];
  const int lane = lane_id();
  const int wave = wave_id();
  const int W = blockDim.x >> 6;
  const int tile = blockIdx.x;
  const int cw0 = tile * TW;
  const int nvalid = min(TW, B - cw0);
  const TileState st = tile_state(wsE0, wsE1, wsM, wsR, wsZ, g, tile);

  ingest_tile<DV>(g, llr32, llr64, cw0, nvalid, st, stage, wave, W, lane);

  bool active = lane < nvalid;
  int my_iters = 0;
  for (int it = 0;; ++it) {
    float *En = ((it + 1) & 1) ? st.E1 : st.E0;  // receives E^(it+1)
    int unsat = 0;
    for (int c = wave; c < g.m; c += W) {
      int e0, dc;
      check_range<DC>(g, c, e0, dc);
      unsat |= check_update<DC>(st.M, En, st.Z, g.col_idx, e0, dc, lane, active);
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
    for (int v = wave; v < g.n; v += W) {
      int p0, dv;
      var_range<DV>(g, v, p0, dv);
      var_update<DV>(st.R, En, st.M, st.Z, g.var_edges, p0, dv, v, lane, active);
    }
    __syncthreads();
  }

  egress_tile<DV>(g, st, my_iters, cw0, nvalid, post, hard, stage, wave, W, lane);
  if (wave == 0 && lane < nvalid) iters[cw0 + lane] = my_iters;
}

}  // namespace ldpc

using namespace ldpc;

size_t plain_workspace_bytes(const ldpc_graph_s *g, int32_t batch) {
  const size_t tiles = ((size_t)batch + TW - 1) / TW;
  return 3 * align256(tiles * (size_t)g->nnz * TW * sizeof(float)) +
         align256(tiles * (size_t)g->n * TW * sizeof(float)) + align256(tiles * (size_t)g->n * 8);
}

namespace {

using PlainKernel = void (*)(GraphDev, const float *, const double *, int, int, int, float *, float *, float *,
                             float *, unsigned long long *, uint8_t *, float *, int32_t *);

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
  const size_t ebytes = align256(tiles * (size_t)g->nnz * TW * sizeof(float));
  float *wsE0 = (float *)p;
  float *wsE1 = (float *)(p + ebytes);
  float *wsM = (float *)(p + 2 * ebytes);
  p += 3 * ebytes;
  float *wsR = (float *)p;
  p += align256(tiles * (size_t)g->n * TW * sizeof(float));
  unsigned long long *wsZ = (unsigned long long *)p;
  PlainKernel k = pick_plain(g, d);
  const float *l32 = llr_f64 ? nullptr : (const float *)llr;
  const double *l64 = llr_f64 ? (const double *)llr : nullptr;
  hipLaunchKernelGGL(k, dim3((unsigned)tiles), dim3(64 * waves), 0, stream, d, l32, l64, (int)batch, (int)max_iters,
                     (int)(early_stop != 0), wsE0, wsE1, wsM, wsR, wsZ, hard, post, iters);
  LDPC_HIP_CHECK(hipGetLastError());
  return LDPC_OK;
}
