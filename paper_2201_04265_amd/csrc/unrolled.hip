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

// Factors of the check rule's derivative for one edge, from what the check rule
// computed anyway: q = e^-|m| of the incoming message m and r = e^|E| of the outgoing E.
//   tau   = tanh(m/2)    = sign(m) (1 - q) / (1 + q), with 1 - q = 1 - e^-x from its
//                          Taylor series x (1 - x/2 + x^2/6 - x^3/24 + x^4/120) when
//                          x = |m| < 0.15 (no cancellation)
//   sech2 = sech^2(m/2)  = 4 q / (1 + q)^2          (no 1 - tanh^2 cancellation)
//   cosh2 = cosh^2(E/2)  = (r + 1)^2 / (4 r)
__device__ __forceinline__ void adjoint_factors(float m, float q, float r, float &tau, float &sech2, float &cosh2) {
  const float x = fabsf(m);
  float t = fmaf(x, 1.0f / 120.0f, -1.0f / 24.0f);
  t = fmaf(x, t, 1.0f / 6.0f);
  t = fmaf(x, t, -0.5f);
  t = fmaf(x, t, 1.0f);
  const float u = x < 0.15f ? x * t : 1.0f - q;
  const float ip = __builtin_amdgcn_rcpf(1.0f + q);
  tau = copysignf(u * ip, m);
  sech2 = 4.0f * q * ip * ip;
  const float rp = r + 1.0f;
  cosh2 = 0.25f * rp * rp * __builtin_amdgcn_rcpf(r);
}

// Sum over the 64 lanes in a fixed butterfly order (same result in every lane).
__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// Adjoint of the check rule for one check, given a_i = dE_i cosh^2(E_i/2),
// tau_u = tanh(M_u/2) and sech2_j = sech^2(M_j/2): emits dA_j = [-20 <= A_j <= 20]
// sech2_j sum_{i != j} a_i prod_{u != i, j} tau_u, with the inner sum from prefix and
// suffix pairs (P, S).
template <int DC, typename Emit>
__device__ __forceinline__ void check_adjoint(const float *av, const float *sech2, const float *tau, const float *a,
                                              int dc, Emit &&emit) {
  constexpr int DCM = DC > 0 ? DC : -DC;
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
      const float dm = sech2[j] * sx;
      emit(j, (av[j] >= -kLmax && av[j] <= kLmax) ? dm : 0.0f);
      S = S * tau[j] + a[j] * P;
      P = P * tau[j];
    }
  }
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
      double x[DVM];
      int eid[DVM];
      const float r = st.R[v * TW + lane];
      double L = (double)r;  // the plain decoder's FP64 sums (var_total) over weighted messages
#pragma unroll
      for (int j = 0; j < DVM; ++j) {
        if (DV > 0 || j < dv) {
          eid[j] = g.var_edges[p0 + j];
          x[j] = (double)wt[eid[j]] * (double)st.E[eid[j] * TW + lane];  // exact product
          L += x[j];
        }
      }
      if (t < T) {
#pragma unroll
        for (int j = 0; j < DVM; ++j)
          if (DV > 0 || j < dv) An[eid[j] * TW + lane] = (float)(L - x[j]);
      } else {
        st.R[v * TW + lane] = (float)L;  // posterior replaces R after the last iteration
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
      float av[DCM], mv[DCM], ev[DCM], tau[DCM], a[DCM], sh[DCM], qv[DCM], rv[DCM];
#pragma unroll
      for (int j = 0; j < DCM; ++j) {
        if (DC > 0 || j < dc) {
          av[j] = At[(e0 + j) * TW + lane];
          mv[j] = clamp_msg(av[j]);
        }
      }
      check_core<DC, false, true>(mv, dc, ev, qv, rv);  // E^(t), recomputed exactly as in the forward
#pragma unroll
      for (int j = 0; j < DCM; ++j) {
        if (DC > 0 || j < dc) {
          const float gg = st.G[(e0 + j) * TW + lane];
          const float s = wave_sum(gg * ev[j]);
          if (lane == 0) wpt[e0 + j] = s;
          float ch;
          adjoint_factors(mv[j], qv[j], rv[j], tau[j], sh[j], ch);
          a[j] = gg * wt[e0 + j] * ch;
        }
      }
      check_adjoint<DC>(av, sh, tau, a, dc, [&](int j, float da) { st.D[(e0 + j) * TW + lane] = da; });
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

// ---- LDS form: one word per workgroup -------------------------------------------
//
// For codes whose per-word state fits in LDS the same iterations run with the word's
// messages on chip, one word per workgroup (threads take checks, then variables, in
// Algorithm 1's interleave), so HBM carries only the LLRs, the weights, the outputs and
// the checkpoints.  Same operations in the same order per word as the tile kernels:
// the forward's outputs are identical to theirs (and, with all weights 1, to the plain
// decoder's).  Checkpoints are [word][t][E] (A^(t)), written by the check phase that
// reads them.  In the backward each workgroup takes K consecutive words and adds their
// weight gradients, in word order, into its own [T][E] row of the workspace; the rows
// are then summed in a fixed order (reduce_rows): deterministic, K fixed by the batch size.

__host__ __device__ inline size_t unrolled_lds_bwd_bytes(int64_t nnz, int32_t n) {
  return (size_t)nnz * 4 + (size_t)n * 4 + 16;
}
// Forward: the messages, plus the current iteration's weight row when it fits too
// (staged once per iteration by coalesced reads instead of gathered per edge).
__host__ __device__ inline size_t unrolled_lds_fwd_bytes(int64_t nnz, bool stage_w) {
  return (size_t)nnz * (stage_w ? 8 : 4) + 16;
}
// Words per backward workgroup: a function of the batch only, so that the summation
// order of the weight gradients does not depend on the device.
__host__ __device__ inline int unrolled_lds_words_per_group(int32_t batch) {
  return batch <= 2048 ? 1 : (batch + 2047) / 2048;
}

template <int DC, int DV, bool STAGE_W>
__global__ void __launch_bounds__(512)
    unrolled_fwd_lds(GraphDev g, const float *__restrict__ llr, const float *__restrict__ w, int B, int T,
                     float *__restrict__ ckpt, float *__restrict__ post) {
  constexpr int DVM = DV > 0 ? DV : -DV;
  constexpr int DCM = DC > 0 ? DC : -DC;
  extern __shared__ __align__(16) float smem[];
  float *X = smem;                 // A^(t) before the check phase, E^(t) after it
  float *Wl = smem + g.nnz;        // weight row of the iteration (when staged)
  const int tid = threadIdx.x, NT = blockDim.x;
  const int word = blockIdx.x;
  const size_t n = (size_t)g.n, E = (size_t)g.nnz;
  const float *R = llr + (size_t)word * n;
  float *out = post + (size_t)word * n;
  for (int v = tid; v < g.n; v += NT) {  // A^(1) = R on every edge
    int p0, dv;
    var_range<DV>(g, v, p0, dv);
    const float r = R[v];
    for (int j = 0; j < dv; ++j) X[g.var_edges[p0 + j]] = r;
    if (T == 0) out[v] = r;
  }
  lds_barrier();
  for (int t = 1; t <= T; ++t) {
    float *Ck = ckpt + ((size_t)word * T + (t - 1)) * E;
    for (int c = tid; c < g.m; c += NT) {
      int e0, dc;
      check_range<DC>(g, c, e0, dc);
      float av[DCM], mv[DCM], ev[DCM];
      lds_row_load<DC>(X + e0, dc, av);
#pragma unroll
      for (int j = 0; j < DCM; ++j) {
        if (DC > 0 || j < dc) {
          Ck[e0 + j] = av[j];
          mv[j] = clamp_msg(av[j]);
        }
      }
      check_core<DC>(mv, dc, ev);
      lds_row_store<DC>(X + e0, dc, ev);
    }
    const float *wt = w + (size_t)(t - 1) * E;
    if (STAGE_W)
      for (int e = tid; e < g.nnz; e += NT) Wl[e] = wt[e];
    lds_barrier();
    for (int v = tid; v < g.n; v += NT) {
      int p0, dv;
      var_range<DV>(g, v, p0, dv);
      double x[DVM];
      int eid[DVM];
      double L = (double)R[v];  // the plain decoder's FP64 sums (var_total) over weighted messages
#pragma unroll
      for (int j = 0; j < DVM; ++j) {
        if (DV > 0 || j < dv) {
          eid[j] = g.var_edges[p0 + j];
          x[j] = (double)(STAGE_W ? Wl[eid[j]] : wt[eid[j]]) * (double)X[eid[j]];  // exact product
          L += x[j];
        }
      }
      if (t < T) {
#pragma unroll
        for (int j = 0; j < DVM; ++j)
          if (DV > 0 || j < dv) X[eid[j]] = (float)(L - x[j]);
      } else {
        out[v] = (float)L;
      }
    }
    lds_barrier();
  }
}

template <int DC, int DV>
__global__ void __launch_bounds__(512)
    unrolled_bwd_lds(GraphDev g, const float *__restrict__ w, int B, int T, int K, const float *__restrict__ ckpt,
                     const float *__restrict__ gpost, float *__restrict__ wpart, float *__restrict__ grad_llr) {
  constexpr int DVM = DV > 0 ? DV : -DV;
  constexpr int DCM = DC > 0 ? DC : -DC;
  extern __shared__ __align__(16) float smem[];
  float *X = smem;        // G^(t) before the check phase, dA^(t) after it
  float *dR = X + g.nnz;  // d loss / d R of the word
  const int tid = threadIdx.x, NT = blockDim.x;
  const size_t n = (size_t)g.n, E = (size_t)g.nnz;
  float *wp = wpart + (size_t)blockIdx.x * (size_t)T * E;
  for (int k = 0; k < K; ++k) {
    const int word = blockIdx.x * K + k;
    if (word >= B) break;  // same in every thread
    const float *gL = gpost + (size_t)word * n;
    for (int v = tid; v < g.n; v += NT) {  // G^(T) = gL on every edge of v, dR = gL
      int p0, dv;
      var_range<DV>(g, v, p0, dv);
      const float gl = gL[v];
      dR[v] = gl;
      for (int j = 0; j < dv; ++j) X[g.var_edges[p0 + j]] = gl;
    }
    lds_barrier();
    // The global inputs of a thread's first check (its checkpoint row, weights and
    // weight-gradient row) are fetched one iteration ahead, during the variable phase.
    float nav[DCM], nwt[DCM], nwp[DCM];
    auto fetch = [&](int tt) {
      if (tid >= g.m || tt < 1) return;
      int e0, dc;
      check_range<DC>(g, tid, e0, dc);
      const size_t off = (size_t)(tt - 1) * E + (size_t)e0;
#pragma unroll
      for (int j = 0; j < DCM; ++j) {
        if (DC > 0 || j < dc) {
          nav[j] = ckpt[(size_t)word * T * E + off + j];
          nwt[j] = w[off + j];
          nwp[j] = k == 0 ? 0.0f : wp[off + j];
        }
      }
    };
    fetch(T);
    for (int t = T; t >= 1; --t) {
      const float *Ck = ckpt + ((size_t)word * T + (t - 1)) * E;
      const float *wt = w + (size_t)(t - 1) * E;
      float *wpt = wp + (size_t)(t - 1) * E;
      for (int c = tid; c < g.m; c += NT) {
        int e0, dc;
        check_range<DC>(g, c, e0, dc);
        const bool first = c == tid;
        float av[DCM], mv[DCM], ev[DCM], tau[DCM], a[DCM], gg[DCM], sh[DCM], qv[DCM], rv[DCM], wv[DCM], old[DCM];
#pragma unroll
        for (int j = 0; j < DCM; ++j) {
          if (DC > 0 || j < dc) {
            av[j] = first ? nav[j] : Ck[e0 + j];
            wv[j] = first ? nwt[j] : wt[e0 + j];
            old[j] = first ? nwp[j] : (k == 0 ? 0.0f : wpt[e0 + j]);
            mv[j] = clamp_msg(av[j]);
          }
        }
        check_core<DC, false, true>(mv, dc, ev, qv, rv);  // E^(t), recomputed exactly as in the forward
        lds_row_load<DC>(X + e0, dc, gg);
#pragma unroll
        for (int j = 0; j < DCM; ++j) {
          if (DC > 0 || j < dc) {
            const float contrib = gg[j] * ev[j];
            wpt[e0 + j] = k == 0 ? contrib : old[j] + contrib;
            float ch;
            adjoint_factors(mv[j], qv[j], rv[j], tau[j], sh[j], ch);
            a[j] = gg[j] * wv[j] * ch;
          }
        }
        check_adjoint<DC>(av, sh, tau, a, dc, [&](int j, float da) { X[e0 + j] = da; });
      }
      lds_barrier();
      fetch(t - 1);
      for (int v = tid; v < g.n; v += NT) {
        int p0, dv;
        var_range<DV>(g, v, p0, dv);
        float dv_[DVM], pre[DVM];
        int eid[DVM];
#pragma unroll
        for (int j = 0; j < DVM; ++j) {
          if (DV > 0 || j < dv) {
            eid[j] = g.var_edges[p0 + j];
            dv_[j] = X[eid[j]];
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
        dR[v] += acc;
        if (t > 1) {
          float suf = 0.0f;
#pragma unroll
          for (int j = DVM - 1; j >= 0; --j) {
            if (DV > 0 || j < dv) {
              X[eid[j]] = pre[j] + suf;
              suf += dv_[j];
            }
          }
        }
      }
      lds_barrier();
    }
    for (int v = tid; v < g.n; v += NT) grad_llr[(size_t)word * n + v] = dR[v];
    lds_barrier();  // dR and X are reused by the next word
  }
}

// grad_w[i] = sum of the rows' partials wpart[r][i] in a fixed order: rows are summed in
// ascending order within chunks of kReduceChunk, then the chunk sums in ascending order
// (one pass when there is a single chunk).  Deterministic for a given row count.
constexpr int kReduceChunk = 32;

__global__ void reduce_rows_chunks(const float *__restrict__ wpart, int rows, size_t len, float *__restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  const int r0 = blockIdx.y * kReduceChunk, r1 = min(rows, r0 + kReduceChunk);
  float s = 0.0f;
  for (int r = r0; r < r1; ++r) s += wpart[(size_t)r * len + i];
  out[(size_t)blockIdx.y * len + i] = s;
}

inline size_t reduce_part_bytes(int rows, size_t len) {
  const size_t chunks = ((size_t)rows + kReduceChunk - 1) / kReduceChunk;
  return chunks > 1 ? chunks * len * sizeof(float) : 0;
}

// part: reduce_part_bytes(rows, len) bytes of scratch.  rows == 0 writes zeros.
ldpc_status reduce_rows(const float *wpart, int rows, size_t len, float *part, float *out, hipStream_t stream) {
  const unsigned cols = (unsigned)((len + 255) / 256);
  const int chunks = (rows + kReduceChunk - 1) / kReduceChunk;
  if (chunks <= 1) {
    hipLaunchKernelGGL(reduce_rows_chunks, dim3(cols, 1), dim3(256), 0, stream, wpart, rows, len, out);
    LDPC_HIP_CHECK(hipGetLastError());
    return LDPC_OK;
  }
  hipLaunchKernelGGL(reduce_rows_chunks, dim3(cols, (unsigned)chunks), dim3(256), 0, stream, wpart, rows, len, part);
  LDPC_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(reduce_rows_chunks, dim3(cols, 1), dim3(256), 0, stream, (const float *)part, chunks, len, out);
  LDPC_HIP_CHECK(hipGetLastError());
  return LDPC_OK;
}

}  // namespace ldpc

using namespace ldpc;

namespace {

// Largest dynamic LDS one workgroup of the graph's device may use (queried once).
int lds_limit(ldpc_graph_s *g) {
  std::lock_guard<std::mutex> lock(g->stream_mu);
  if (g->lds_limit == 0) {
    int dev = 0, lim = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess)
      g->lds_limit = lim;
  }
  return g->lds_limit;
}

// The LDS form runs when a word's backward state (4E + 4n bytes) fits one workgroup.
bool use_lds_form(ldpc_graph_s *g) { return unrolled_lds_bwd_bytes(g->nnz, g->n) + 64 <= (size_t)lds_limit(g); }

int lds_form_threads(const ldpc_graph_s *g) {
  const int big = std::max(g->m, g->n);
  int nt = 64;
  while (nt < 512 && nt < big) nt *= 2;
  return nt;
}

}  // namespace

extern "C" ldpc_status ldpc_unrolled_sizes(ldpc_graph_t g, int32_t batch, int32_t T, size_t *ckpt_bytes,
                                           size_t *fwd_ws_bytes, size_t *bwd_ws_bytes) {
  if (!g) return set_error(LDPC_ERR_INVALID_ARG, "graph is NULL");
  if (batch < 0 || T < 0) return set_error(LDPC_ERR_INVALID_ARG, "negative batch or T");
  if (use_lds_form(g)) {
    const size_t groups = ((size_t)batch + unrolled_lds_words_per_group(batch) - 1) /
                          (size_t)unrolled_lds_words_per_group(batch);
    const size_t len = (size_t)T * (size_t)g->nnz;
    if (ckpt_bytes) *ckpt_bytes = al256((size_t)batch * len * 4);
    if (fwd_ws_bytes) *fwd_ws_bytes = 256;
    if (bwd_ws_bytes) *bwd_ws_bytes = al256(groups * len * 4) + al256(reduce_part_bytes((int)groups, len)) + 256;
    return LDPC_OK;
  }
  const size_t tiles = ((size_t)batch + TW - 1) / TW;
  const size_t len = (size_t)T * (size_t)g->nnz;
  if (ckpt_bytes) *ckpt_bytes = tiles * unrolled_ckpt_tile(g->nnz, T);
  if (fwd_ws_bytes) *fwd_ws_bytes = tiles * unrolled_ws_tile(g->nnz, g->n);
  if (bwd_ws_bytes)
    *bwd_ws_bytes = tiles * unrolled_ws_tile(g->nnz, g->n) + al256(tiles * len * 4) +
                    al256(reduce_part_bytes((int)tiles, len));
  return LDPC_OK;
}

namespace {
using FwdKernel = void (*)(GraphDev, const float *, const float *, int, int, char *, char *, float *);
using BwdKernel = void (*)(GraphDev, const float *, int, int, const char *, const float *, char *, float *,
                           float *);
using LdsFwdKernel = void (*)(GraphDev, const float *, const float *, int, int, float *, float *);
using LdsBwdKernel = void (*)(GraphDev, const float *, int, int, int, const float *, const float *, float *, float *);

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
  if (use_lds_form(g)) {
    const bool stage_w = unrolled_lds_fwd_bytes(g->nnz, true) + 64 <= (size_t)lds_limit(g);
    LdsFwdKernel kl = nullptr;
#define LDPC_PICK(C, V) kl = stage_w ? unrolled_fwd_lds<C, V, true> : unrolled_fwd_lds<C, V, false>
    LDPC_KIND_SWITCH(kernel_kind(g), LDPC_PICK)
#undef LDPC_PICK
    const size_t lds = unrolled_lds_fwd_bytes(g->nnz, stage_w);
    if (lds > 65536)
      LDPC_HIP_CHECK(hipFuncSetAttribute((const void *)kl, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kl, dim3((unsigned)batch), dim3(lds_form_threads(g)), lds, stream, graph_dev(g), llr, w,
                       (int)batch, (int)T, (float *)ckpt, posterior);
    LDPC_HIP_CHECK(hipGetLastError());
    return LDPC_OK;
  }
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
    if (T > 0) return reduce_rows(nullptr, 0, (size_t)T * (size_t)g->nnz, nullptr, grad_w, stream);
    return LDPC_OK;
  }
  st = check_buffers(batch, T, grad_post, grad_llr, w, workspace, ws_bytes, bw, ckpt, ckpt_bytes, ck);
  if (st != LDPC_OK) return st;
  if (use_lds_form(g)) {
    LdsBwdKernel kl = nullptr;
#define LDPC_PICK(C, V) kl = unrolled_bwd_lds<C, V>
    LDPC_KIND_SWITCH(kernel_kind(g), LDPC_PICK)
#undef LDPC_PICK
    const size_t lds = unrolled_lds_bwd_bytes(g->nnz, g->n);
    if (lds > 65536)
      LDPC_HIP_CHECK(hipFuncSetAttribute((const void *)kl, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const int K = unrolled_lds_words_per_group(batch);
    const int groups = (batch + K - 1) / K;
    const size_t len = (size_t)T * (size_t)g->nnz;
    float *wpart = (float *)workspace;
    float *part = (float *)((char *)workspace + al256((size_t)groups * len * 4));
    hipLaunchKernelGGL(kl, dim3((unsigned)groups), dim3(lds_form_threads(g)), lds, stream, graph_dev(g), w,
                       (int)batch, (int)T, K, (const float *)ckpt, grad_post, wpart, grad_llr);
    LDPC_HIP_CHECK(hipGetLastError());
    if (T > 0) return reduce_rows(wpart, groups, len, part, grad_w, stream);
    return LDPC_OK;
  }
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
    float *part = (float *)((char *)wpart + al256((size_t)tiles * len * 4));
    return reduce_rows(wpart, tiles, len, part, grad_w, stream);
  }
  return LDPC_OK;
}
