// Differentiable form: unrolled per-edge-weighted flooding iterations and their adjoint.
//
// Forward, per word (T iterations, no early stop; Eqs. 5-7 with a weight on every
// c->v message where it enters a variable-node sum):
//   A^(1)_e   = R_v
//   E^(t)_e   = check rule of Eq. 5 on M^(t) = clamp(A^(t), -20, 20)
//   A^(t+1)_e = R_v + sum_{e' in N(v), e' != e} w^(t)_e' E^(t)_e'
//   L_v       = R_v + sum_{e in N(v)} w^(T)_e E^(T)_e
// With all weights 1 this is the plain decoder run for T iterations without early
// stop, operation for operation (x * 1 is exact), so the posteriors agree bit for bit.
// The forward checkpoints A^(t) for every t (the v->c messages, pre-clamp); the
// backward recomputes the check messages from them instead of storing them.
//
// Backward, given gL = d loss / d L, t = T..1, with G^(t) = d loss / d (w^(t) E^(t)):
//   G^(T)_e = gL_v,  dR_v = gL_v
//   dw^(t)_e = sum over words of G^(t)_e E^(t)_e          (per tile, then over tiles in order)
//   dE^(t)_e = G^(t)_e w^(t)_e
//   dM^(t)_j = sum_{i != j} dE_i dE_i/dM_j,  dE_i/dM_j = cosh^2(E_i/2) sech^2(M_j/2) prod_{u != i,j} tanh(M_u/2)
//   dA^(t)_j = dM^(t)_j [ -20 <= A^(t)_j <= 20 ]
//   dR_v += sum_{e in N(v)} dA^(t)_e,   G^(t-1)_e = sum_{e' in N(v), e' != e} dA^(t)_e'
// The inner sum over i != j is done in O(dc) with prefix/suffix pairs
// (P, S) = (prod tau, sum_i a_i prod_{u != i} tau_u), combined as
// (P1 P2, S1 P2 + S2 P1), where a_i = dE_i cosh^2(E_i/2) and tau_u = tanh(M_u/2).
// Reductions run in a fixed order: no floating-point atomics.
#include "internal.h"
#include "tile.h"

namespace ldpc {

// sech^2(x/2) = 4q / (1+q)^2 and cosh^2(x/2) = (1+q)^2 / (4q) with q = e^-|x|
// (no 1 - tanh^2 cancellation).
__device__ __forceinline__ float sech2_half(float x) {
  const float q = expf(-fabsf(x));
  const float d = 1.0f + q;
  return 4.0f * q / (d * d);
}
__device__ __forceinline__ float cosh2_half(float x) {
  const float q = expf(-fabsf(x));
  const float d = 1.0f + q;
  return d * d / (4.0f * q);
}

// Sum over the 64 lanes in a fixed butterfly order (same result in every lane).
__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

struct UnrolledTile {
  float *A;  // [T][nnz][64] checkpoints of the v->c messages, pre-clamp
  float *E;  // [nnz][64] c->v messages of the current iteration (forward)
  float *R;  // [n][64] channel LLRs, then the posterior (forward) / dR (backward)
  float *G;  // [nnz][64] G^(t) (backward)
  float *D;  // [nnz][64] dA^(t) (backward)
};

__host__ __device__ inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }
__host__ __device__ inline size_t unrolled_ckpt_tile(int64_t nnz, int T) {
  return al256((size_t)T * (size_t)nnz * TW * sizeof(float));
}
__host__ __device__ inline size_t unrolled_ws_tile(int64_t nnz, int32_t n) {
  return 2 * al256((size_t)nnz * TW * sizeof(float)) + al256((size_t)n * TW * sizeof(float));
}

// [B][n] rows -> [n][64] columns of a tile through 64 x 64 LDS blocks (x = 0 beyond B).
__device__ __forceinline__ void rows_to_tile(const float *__restrict__ src, int n, int cw0, int nvalid, float *dst,
                                             float (*stage)[TW + 1], int wave, int W, int lane) {
  for (int v0 = 0; v0 < n; v0 += TW) {
    for (int r = wave; r < TW; r += W) {
      const int v = v0 + lane;
      stage[r][lane] = (r < nvalid && v < n) ? src[(size_t)(cw0 + r) * (size_t)n + (size_t)v] : 0.0f;
    }
    __syncthreads();
    for (int q = wave; q < TW && v0 + q < n; q += W) dst[(v0 + q) * TW + lane] = stage[lane][q];
    __syncthreads();
  }
}

__device__ __forceinline__ void tile_to_rows(const float *src, int n, int cw0, int nvalid, float *__restrict__ dst,
                                             float (*stage)[TW + 1], int wave, int W, int lane) {
  for (int v0 = 0; v0 < n; v0 += TW) {
    for (int q = wave; q < TW && v0 + q < n; q += W) stage[q][lane] = src[(v0 + q) * TW + lane];
    __syncthreads();
    for (int r = wave; r < nvalid; r += W) {
      const int v = v0 + lane;
      if (v < n) dst[(size_t)(cw0 + r) * (size_t)n + (size_t)v] = stage[lane][r];
    }
    __syncthreads();
  }
}

template <int DC, int DV>
__global__ void __launch_bounds__(512)
    unrolled_fwd_kernel(GraphDev g, const float *__restrict__ llr, const float *__restrict__ w, int B, int T,
                        char *ckpt, char *ws, float *__restrict__ post) {
  constexpr int DVM = DV > 0 ? DV : -DV;
  constexpr int DCM = DC > 0 ? DC : -DC;
  __shared__ float stage[TW][TW + 1];
  const int lane = lane_id(), wave = wave_id(), W = blockDim.x >> 6;
  const int tile = blockIdx.x, cw0 = tile * TW, nvalid = min(TW, B - cw0);
  const size_t esz = (size_t)g.nnz * TW;
  UnrolledTile st;
  st.A = (float *)(ckpt + (size_t)tile * unrolled_ckpt_tile(g.nnz, T));
  char *wb = ws + (size_t)tile * unrolled_ws_tile(g.nnz, g.n);
  st.E = (float *)wb;
  st.R = (float *)(wb + 2 * al256(esz * sizeof(float)));

  rows_to_tile(llr, g.n, cw0, nvalid, st.R, stage, wave, W, lane);
  if (T > 0) {
    for (int v = wave; v < g.n; v += W) {  // A^(1) = R on every edge
      int p0, dv;
      var_range<DV>(g, v, p0, dv);
      const float r = st.R[v * TW + lane];
      for (int j = 0; j < dv; ++j) st.A[g.var_edges[p0 + j] * TW + lane] = r;
    }
  }
  __syncthreads();

  for (int t = 1; t <= T; ++t) {
    const float *At = st.A + (size_t)(t - 1) * esz;
    for (int c = wave; c < g.m; c += W) {
      int e0, dc;
      check_range<DC>(g, c, e0, dc);
      float mv[DCM], ev[DCM];
#pragma unroll
      for (int j = 0; j < DCM; ++j)
        if (DC > 0 || j < dc) mv[j] = clamp_msg(At[(e0 + j) * TW + lane]);
      check_core<DC>(mv, dc, ev);
#pragma unroll
      for (int j = 0; j < DCM; ++j)
        if (DC > 0 || j < dc) st.E[(e0 + j) * TW + lane] = ev[j];
    }
    __syncthreads();
    const float *wt = w + (size_t)(t - 1) * (size_t)g.nnz;
    float *An = st.A + (size_t)t * esz;  // A^(t+1), written when t < T
    for (int v = wave; v < g.n; v += W) {
      int p0, dv;
      var_range<DV>(g, v, p0, dv);
      float ev[DVM], pre[DVM];
      int eid[DVM];
      const float r = st.R[v * TW + lane];
#pragma unroll
      for (int j = 0; j < DVM; ++j) {
        if (DV > 0 || j < dv) {
          eid[j] = g.var_edges[p0 + j];
          ev[j] = wt[eid[j]] * st.E[eid[j] * TW + lane];
        }
      }
      float acc = r;
#pragma unroll
      for (int j = 0; j < DVM; ++j) {
        if (DV > 0 || j < dv) {
          pre[j] = acc;
          acc += ev[j];
        }
      }
      if (t < T) {
        var_exclusive<DV>(pre, ev, dv, [&](int j, float x) { An[eid[j] * TW + lane] = x; });
      } else {
        st.R[v * TW + lane] = acc;  // posterior replaces R after the last iteration
      }
    }
    __syncthreads();
  }
  tile_to_rows(st.R, g.n, cw0, nvalid, post, stage, wave, W, lane);
}

template <int DC, int DV>
__global__ void __launch_bounds__(512)
    unrolled_bwd_kernel(GraphDev g, const float *__restrict__ w, int B, int T, const char *ckpt,
                        const float *__restrict__ gpost, char *ws, float *__restrict__ wpart,
                        float *__restrict__ grad_llr) {
  constexpr int DVM = DV > 0 ? DV : -DV;
  constexpr int DCM = DC > 0 ? DC : -DC;
  __shared__ float stage[TW][TW + 1];
  const int lane = lane_id(), wave = wave_id(), W = blockDim.x >> 6;
  const int tile = blockIdx.x, cw0 = tile * TW, nvalid = min(TW, B - cw0);
  const size_t esz = (size_t)g.nnz * TW;
  UnrolledTile st;
  st.A = (float *)(ckpt + (size_t)tile * unrolled_ckpt_tile(g.nnz, T));
  char *wb = ws + (size_t)tile * unrolled_ws_tile(g.nnz, g.n);
  st.G = (float *)wb;
  st.D = (float *)(wb + al256(esz * sizeof(float)));
  st.R = (float *)(wb + 2 * al256(esz * sizeof(float)));
  float *wp = wpart + (size_t)tile * (size_t)T * (size_t)g.nnz;

  rows_to_tile(gpost, g.n, cw0, nvalid, st.R, stage, wave, W, lane);  // dR = gL
  for (int v = wave; v < g.n; v += W) {                                // G^(T) = gL on every edge of v
    int p0, dv;
    var_range<DV>(g, v, p0, dv);
    const float gl = st.R[v * TW + lane];
    for (int j = 0; j < dv; ++j) st.G[g.var_edges[p0 + j] * TW + lane] = gl;
  }
  __syncthreads();

  for (int t = T; t >= 1; --t) {
    const float *At = st.A + (size_t)(t - 1) * esz;
    const float *wt = w + (size_t)(t - 1) * (size_t)g.nnz;
    float *wpt = wp + (size_t)(t - 1) * (size_t)g.nnz;
    for (int c = wave; c < g.m; c += W) {
      int e0, dc;
      check_range<DC>(g, c, e0, dc);
      float av[DCM], mv[DCM], ev[DCM], tau[DCM], a[DCM];
#pragma unroll
      for (int j = 0; j < DCM; ++j) {
        if (DC > 0 || j < dc) {
          av[j] = At[(e0 + j) * TW + lane];
          mv[j] = clamp_msg(av[j]);
        }
      }
      check_core<DC>(mv, dc, ev);  // E^(t), recomputed exactly as in the forward
#pragma unroll
      for (int j = 0; j < DCM; ++j) {
        if (DC > 0 || j < dc) {
          const float gg = st.G[(e0 + j) * TW + lane];
          const float s = wave_sum(gg * ev[j]);
          if (lane == 0) wpt[e0 + j] = s;
          a[j] = gg * wt[e0 + j] * cosh2_half(ev[j]);
          tau[j] = tanhf(0.5f * mv[j]);
        }
      }
      // prefix pairs over items < j, then suffix pairs over items > j
      float pP[DCM], pS[DCM];
      float P = 1.0f, S = 0.0f;
#pragma unroll
      for (int j = 0; j < DCM; ++j) {
        if (DC > 0 || j < dc) {
          pP[j] = P;
          pS[j] = S;
          S = S * tau[j] + a[j] * P;
          P = P * tau[j];
        }
      }
      P = 1.0f;
      S = 0.0f;
#pragma unroll
      for (int j = DCM - 1; j >= 0; --j) {
        if (DC > 0 || j < dc) {
          const float sx = pS[j] * P + S * pP[j];
          const float dm = sech2_half(mv[j]) * sx;
          const float da = (av[j] >= -kLmax && av[j] <= kLmax) ? dm : 0.0f;
          st.D[(e0 + j) * TW + lane] = da;
          S = S * tau[j] + a[j] * P;
          P = P * tau[j];
        }
      }
    }
    __syncthreads();
    for (int v = wave; v < g.n; v += W) {
      int p0, dv;
      var_range<DV>(g, v, p0, dv);
      float dv_[DVM], pre[DVM];
      int eid[DVM];
#pragma unroll
      for (int j = 0; j < DVM; ++j) {
        if (DV > 0 || j < dv) {
          eid[j] = g.var_edges[p0 + j];
          dv_[j] = st.D[eid[j] * TW + lane];
        }
      }
      float acc = 0.0f;
#pragma unroll
      for (int j = 0; j < DVM; ++j) {
        if (DV > 0 || j < dv) {
          pre[j] = acc;
          acc += dv_[j];
        }
      }
      st.R[v * TW + lane] += acc;
      if (t > 1) {
        float suf = 0.0f;
#pragma unroll
        for (int j = DVM - 1; j >= 0; --j) {
          if (DV > 0 || j < dv) {
            st.G[eid[j] * TW + lane] = pre[j] + suf;
            suf += dv_[j];
          }
        }
      }
    }
    __syncthreads();
  }
  tile_to_rows(st.R, g.n, cw0, nvalid, grad_llr, stage, wave, W, lane);
}

// grad_w[i] = sum over tiles (ascending) of the per-tile partials.
__global__ void reduce_tiles(const float *__restrict__ wpart, int tiles, size_t len, float *__restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  float s = 0.0f;
  for (int k = 0; k < tiles; ++k) s += wpart[(size_t)k * len + i];
  out[i] = s;
}

}  // namespace ldpc

using namespace ldpc;

extern "C" ldpc_status ldpc_unrolled_sizes(ldpc_graph_t g, int32_t batch, int32_t T, size_t *ckpt_bytes,
                                           size_t *fwd_ws_bytes, size_t *bwd_ws_bytes) {
  if (!g) return set_error(LDPC_ERR_INVALID_ARG, "graph is NULL");
  if (batch < 0 || T < 0) return set_error(LDPC_ERR_INVALID_ARG, "negative batch or T");
  const size_t tiles = ((size_t)batch + TW - 1) / TW;
  if (ckpt_bytes) *ckpt_bytes = tiles * unrolled_ckpt_tile(g->nnz, T);
  if (fwd_ws_bytes) *fwd_ws_bytes = tiles * unrolled_ws_tile(g->nnz, g->n);
  if (bwd_ws_bytes)
    *bwd_ws_bytes = tiles * unrolled_ws_tile(g->nnz, g->n) + al256(tiles * (size_t)T * (size_t)g->nnz * 4);
  return LDPC_OK;
}

namespace {
using FwdKernel = void (*)(GraphDev, const float *, const float *, int, int, char *, char *, float *);
using BwdKernel = void (*)(GraphDev, const float *, int, int, const char *, const float *, char *, float *,
                           float *);

ldpc_status check_buffers(int32_t batch, int32_t T, const void *in, const void *out, const void *w, const void *ws,
                          size_t ws_bytes, size_t need_ws, const void *ck, size_t ck_bytes, size_t need_ck) {
  if (batch == 0) return LDPC_OK;
  if (!in || !out || !ws) return set_error(LDPC_ERR_INVALID_ARG, "NULL buffer");
  if (T > 0 && (!w || !ck)) return set_error(LDPC_ERR_INVALID_ARG, "NULL weights or checkpoints");
  if (((uintptr_t)ws & 255) || ((uintptr_t)ck & 255))
    return set_error(LDPC_ERR_INVALID_ARG, "workspace and checkpoints must be 256-byte aligned");
  if (ws_bytes < need_ws) return set_error(LDPC_ERR_INVALID_ARG, "workspace too small");
  if (ck_bytes < need_ck) return set_error(LDPC_ERR_INVALID_ARG, "checkpoint buffer too small");
  return LDPC_OK;
}
}  // namespace

extern "C" ldpc_status ldpc_unrolled_forward(ldpc_graph_t g, const float *llr, const float *w, int32_t batch, int32_t T,
                                             float *posterior, void *ckpt, size_t ckpt_bytes, void *workspace,
                                             size_t ws_bytes, hipStream_t stream) {
  size_t ck = 0, fw = 0;
  ldpc_status st = ldpc_unrolled_sizes(g, batch, T, &ck, &fw, nullptr);
  if (st != LDPC_OK) return st;
  st = check_buffers(batch, T, llr, posterior, w, workspace, ws_bytes, fw, ckpt, ckpt_bytes, ck);
  if (st != LDPC_OK || batch == 0) return st;
  FwdKernel k = nullptr;
#define LDPC_PICK(C, V) k = unrolled_fwd_kernel<C, V>
  LDPC_KIND_SWITCH(kernel_kind(g), LDPC_PICK)
#undef LDPC_PICK
  const int tiles = (batch + TW - 1) / TW;
  hipLaunchKernelGGL(k, dim3(tiles), dim3(512), 0, stream, graph_dev(g), llr, w, (int)batch, (int)T, (char *)ckpt,
                     (char *)workspace, posterior);
  LDPC_HIP_CHECK(hipGetLastError());
  return LDPC_OK;
}

extern "C" ldpc_status ldpc_unrolled_backward(ldpc_graph_t g, const float *w, const void *ckpt, size_t ckpt_bytes,
                                              const float *grad_post, int32_t batch, int32_t T, float *grad_llr,
                                              float *grad_w, void *workspace, size_t ws_bytes, hipStream_t stream) {
  size_t ck = 0, bw = 0;
  ldpc_status st = ldpc_unrolled_sizes(g, batch, T, &ck, nullptr, &bw);
  if (st != LDPC_OK) return st;
  if (T > 0 && !grad_w) return set_error(LDPC_ERR_INVALID_ARG, "grad_w is NULL");
  if (batch == 0) {
    if (T > 0) {
      const size_t len = (size_t)T * (size_t)g->nnz;
      hipLaunchKernelGGL(reduce_tiles, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, stream, nullptr, 0, len,
                         grad_w);
      LDPC_HIP_CHECK(hipGetLastError());
    }
    return LDPC_OK;
  }
  st = check_buffers(batch, T, grad_post, grad_llr, w, workspace, ws_bytes, bw, ckpt, ckpt_bytes, ck);
  if (st != LDPC_OK) return st;
  BwdKernel k = nullptr;
#define LDPC_PICK(C, V) k = unrolled_bwd_kernel<C, V>
  LDPC_KIND_SWITCH(kernel_kind(g), LDPC_PICK)
#undef LDPC_PICK
  const int tiles = (batch + TW - 1) / TW;
  const size_t tail = (size_t)tiles * unrolled_ws_tile(g->nnz, g->n);
  float *wpart = (float *)((char *)workspace + tail);
  hipLaunchKernelGGL(k, dim3(tiles), dim3(512), 0, stream, graph_dev(g), w, (int)batch, (int)T, (const char *)ckpt,
                     grad_post, (char *)workspace, wpart, grad_llr);
  LDPC_HIP_CHECK(hipGetLastError());
  if (T > 0) {
    const size_t len = (size_t)T * (size_t)g->nnz;
    hipLaunchKernelGGL(reduce_tiles, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, stream, wpart, tiles, len,
                       grad_w);
    LDPC_HIP_CHECK(hipGetLastError());
  }
  return LDPC_OK;
}
