// Tile state and per-tile data movement shared by the decoder kernels.
#pragma once

#include "internal.h"
#include "spa_core.h"

namespace ldpc {

// HBM state of one 64-word tile (FP32 [index][64]):
//   M  [nnz]  v->c messages (Eq. 6, clamped), stored with their variable's decision
//   E0/E1 [nnz] c->v messages of even / odd steps (Eq. 5)
//   R  [n]  channel LLRs (Eq. 4)
struct TileState {
  float *E0, *E1, *M, *R;
};

// Bytes of one tile's state, each array 256-byte aligned.
__host__ __device__ inline size_t tile_bytes(int64_t nnz, int32_t n) {
  const size_t e = ((size_t)nnz * TW * sizeof(float) + 255) & ~size_t(255);
  const size_t v = ((size_t)n * TW * sizeof(float) + 255) & ~size_t(255);
  return 3 * e + v;
}

// Tile state carved from one contiguous per-tile block.
__device__ __forceinline__ TileState tile_state_block(char *base, int64_t nnz, int32_t n) {
  const size_t e = ((size_t)nnz * TW * sizeof(float) + 255) & ~size_t(255);
  TileState s;
  s.E0 = (float *)base;
  s.E1 = (float *)(base + e);
  s.M = (float *)(base + 2 * e);
  s.R = (float *)(base + 3 * e);
  return s;
}

template <int DV>
__device__ __forceinline__ void var_range(const GraphDev &g, int v, int &p0, int &dv) {
  if (DV > 0) {
    p0 = v * DV;
    dv = DV;
  } else {
    p0 = ld_graph(g.var_ptr, v);
    dv = ld_graph(g.var_ptr, v + 1) - p0;
  }
}

template <int DC>
__device__ __forceinline__ void check_range(const GraphDev &g, int c, int &e0, int &dc) {
  if (DC > 0) {
    e0 = c * DC;
    dc = DC;
  } else {
    e0 = ld_graph(g.row_ptr, c);
    dc = ld_graph(g.row_ptr, c + 1) - e0;
  }
}

// [B][n] channel LLRs -> R of the tile (through 64 x 64 LDS blocks) and the first
// v->c messages M = clamp(R) on every edge, carrying the channel decisions [R <= 0].
template <int DV>
__device__ __forceinline__ void ingest_tile(const GraphDev &g, const float *__restrict__ llr32,
                                            const double *__restrict__ llr64, int cw0, int nvalid, TileState st,
                                            float (*stage)[TW + 1], int wave, int W, int lane, int chunk0 = 0,
                                            int chunk_step = 1) {
  const int n = g.n;
  for (int v0 = chunk0 * TW; v0 < n; v0 += chunk_step * TW) {  // 64-variable chunks
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
      int p0, dv;
      var_range<DV>(g, v, p0, dv);
      const float mx = v2c_store(x, x <= 0.0f);
      for (int j = 0; j < dv; ++j) st.M[ld_graph(g.var_edges, p0 + j) * TW + lane] = mx;
    }
    __syncthreads();
  }
}

// Caller c->v state [B][nnz] (CSR edge order) -> dst [nnz][64] of the tile, through the
// same 64 x 64 LDS blocks as the LLRs.  Lanes past the batch get zeros.
__device__ __forceinline__ void ingest_edges(const GraphDev &g, const float *__restrict__ src, int cw0, int nvalid,
                                             float *__restrict__ dst, float (*stage)[TW + 1], int wave, int W,
                                             int lane) {
  const int nnz = g.nnz;
  for (int e0 = 0; e0 < nnz; e0 += TW) {
    for (int r = wave; r < TW; r += W) {
      const int e = e0 + lane;
      stage[r][lane] = (r < nvalid && e < nnz) ? src[(size_t)(cw0 + r) * (size_t)nnz + (size_t)e] : 0.0f;
    }
    __syncthreads();
    for (int q = wave; q < TW && e0 + q < nnz; q += W) dst[(e0 + q) * TW + lane] = stage[lane][q];
    __syncthreads();
  }
}

// Each lane's c->v messages of its last iteration (E[my_iters & 1]; zeros for a word that
// stopped at 0 without a starting state) -> dst [B][nnz].
__device__ __forceinline__ void egress_edges(const GraphDev &g, TileState st, int my_iters, bool from_state,
                                             int cw0, int nvalid, float *__restrict__ dst, float (*stage)[TW + 1],
                                             int wave, int W, int lane) {
  const int nnz = g.nnz;
  const float *Eb = (my_iters & 1) ? st.E1 : st.E0;
  const bool zero = my_iters == 0 && !from_state;
  for (int e0 = 0; e0 < nnz; e0 += TW) {
    for (int q = wave; q < TW && e0 + q < nnz; q += W) stage[q][lane] = zero ? 0.0f : Eb[(e0 + q) * TW + lane];
    __syncthreads();
    for (int r = wave; r < nvalid; r += W) {
      const int e = e0 + lane;
      if (e < nnz) dst[(size_t)(cw0 + r) * (size_t)nnz + (size_t)e] = stage[lane][r];
    }
    __syncthreads();
  }
}

// Final posterior of each lane's word from its own E buffer -> post and hard [B][n].
// from_state: the decode started from a given c->v state in E0, so a word that stopped
// at iteration 0 returns the posterior of that state (Eq. 7) instead of R.
template <int DV>
__device__ __forceinline__ void egress_tile(const GraphDev &g, TileState st, int my_iters, int cw0, int nvalid,
                                            float *__restrict__ post, uint8_t *__restrict__ hard,
                                            float (*stage)[TW + 1], int wave, int W, int lane, int chunk0 = 0,
                                            int chunk_step = 1, bool from_state = false) {
  constexpr int DMAX = DV > 0 ? DV : -DV;
  const int n = g.n;
  const float *Eb = (my_iters & 1) ? st.E1 : st.E0;
  for (int v0 = chunk0 * TW; v0 < n; v0 += chunk_step * TW) {  // 64-variable chunks
    for (int q = wave; q < TW && v0 + q < n; q += W) {
      const int v = v0 + q;
      int p0, dv;
      var_range<DV>(g, v, p0, dv);
      float ev[DMAX];
      int eid[DMAX];
      const float r = st.R[v * TW + lane];
      const float L = (float)var_posterior<DV>(r, Eb, g.var_edges, p0, dv, lane, ev, eid);
      stage[q][lane] = (my_iters > 0 || from_state) ? L : r;
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


// A check's messages are contiguous (edge e0 = c * DC for a fixed degree), so a row is
// moved with 16- or 8-byte LDS accesses when DC allows: a check's row then starts on
// a multiple of its access width, and consecutive threads' rows fall on disjoint banks.
template <int DC>
__device__ __forceinline__ void lds_row_load(const float *row, int dc, float *v) {
  if constexpr (DC > 0 && DC % 4 == 0) {
#pragma unroll
    for (int h = 0; h < DC / 4; ++h) {
      const float4 x = reinterpret_cast<const float4 *>(row)[h];
      v[4 * h] = x.x;
      v[4 * h + 1] = x.y;
      v[4 * h + 2] = x.z;
      v[4 * h + 3] = x.w;
    }
  } else if constexpr (DC > 0 && DC % 2 == 0) {
#pragma unroll
    for (int h = 0; h < DC / 2; ++h) {
      const float2 x = reinterpret_cast<const float2 *>(row)[h];
      v[2 * h] = x.x;
      v[2 * h + 1] = x.y;
    }
  } else {
    constexpr int DM = DC > 0 ? DC : -DC;
#pragma unroll
    for (int j = 0; j < DM; ++j)
      if (DC > 0 || j < dc) v[j] = row[j];
  }
}

template <int DC>
__device__ __forceinline__ void lds_row_store(float *row, int dc, const float *v) {
  if constexpr (DC > 0 && DC % 4 == 0) {
#pragma unroll
    for (int h = 0; h < DC / 4; ++h)
      reinterpret_cast<float4 *>(row)[h] = make_float4(v[4 * h], v[4 * h + 1], v[4 * h + 2], v[4 * h + 3]);
  } else if constexpr (DC > 0 && DC % 2 == 0) {
#pragma unroll
    for (int h = 0; h < DC / 2; ++h) reinterpret_cast<float2 *>(row)[h] = make_float2(v[2 * h], v[2 * h + 1]);
  } else {
    constexpr int DM = DC > 0 ? DC : -DC;
#pragma unroll
    for (int j = 0; j < DM; ++j)
      if (DC > 0 || j < dc) row[j] = v[j];
  }
}

}  // namespace ldpc
