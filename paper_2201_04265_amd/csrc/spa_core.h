// Device building blocks of flooding sum-product decoding on gfx950.
//
// Layout: a tile holds kTile = 64 codewords, one per wavefront lane.  Every
// per-edge or per-variable array of a tile is stored [index][64] so that a
// wavefront reading "edge e of all 64 words" touches one contiguous 256-byte
// segment; graph indices are wave-uniform and come through scalar loads.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ldpc {

constexpr int TW = 64;          // words per tile (lanes per wavefront)
constexpr float kLmax = 20.0f;  // saturation of variable-to-check messages

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// phi(x) = log((e^x + 1) / (e^x - 1)) = log1p(2 / expm1(x)) for x >= 0, the
// magnitude map of the tanh rule: 2 atanh(prod tanh(a_i / 2)) = phi(sum phi(a_i)).
// phi(0) = +inf and phi(+inf) = 0, so a zero input message zeroes the others.
// expm1 / log1p keep full relative accuracy for small x and for large x.
__device__ __forceinline__ float phi(float x) { return log1pf(2.0f * __builtin_amdgcn_rcpf(expm1f(x))); }

__device__ __forceinline__ float clamp_msg(float x) { return fminf(fmaxf(x, -kLmax), kLmax); }

// Check-node update (Eq. 5) of one check for the 64 words of a tile.
//   Lt: posterior L [n][64]; Et: c->v messages [nnz][64] (read old, write new).
//   M_j = clamp(L_vj - E_old_j) (E_old taken as 0 when !use_old), then
//   E_j = sign_j * phi(sum_{i != j} phi(|M_i|)) with the exclusive sum built from
//   a prefix and a suffix (no total-minus-self), sign_j = parity of the other signs.
// Returns the parity of the hard decisions [L <= 0] over the check: the
// syndrome bit of the decisions the messages were computed from.
// DC > 0: degree fixed at compile time; DC < 0: any degree up to -DC (runtime dc).
template <int DC>
__device__ __forceinline__ int check_update(const float *__restrict__ Lt, float *__restrict__ Et,
                                            const int32_t *__restrict__ col_idx, int e0, int dc, int lane,
                                            bool use_old, bool store) {
  constexpr int DMAX = DC > 0 ? DC : -DC;
  constexpr bool FIXED = DC > 0;
  float lv[DMAX], eo[DMAX], ph[DMAX], pre[DMAX];
#pragma unroll
  for (int j = 0; j < DMAX; ++j) {
    if (FIXED || j < dc) {
      const int v = col_idx[e0 + j];
      lv[j] = Lt[v * TW + lane];
      eo[j] = Et[(e0 + j) * TW + lane];
    }
  }
  int par = 0;
  uint32_t sg = 0;
#pragma unroll
  for (int j = 0; j < DMAX; ++j) {
    if (FIXED || j < dc) {
      par ^= (lv[j] <= 0.0f) ? 1 : 0;
      const float mm = clamp_msg(use_old ? lv[j] - eo[j] : lv[j]);
      sg |= (mm < 0.0f ? 1u : 0u) << j;
      ph[j] = phi(fabsf(mm));
    }
  }
  float acc = 0.0f;
#pragma unroll
  for (int j = 0; j < DMAX; ++j) {
    if (FIXED || j < dc) {
      pre[j] = acc;
      acc += ph[j];
    }
  }
  const uint32_t tot = (uint32_t)__builtin_popcount(sg) & 1u;
  float suf = 0.0f;
#pragma unroll
  for (int j = DMAX - 1; j >= 0; --j) {
    if (FIXED || j < dc) {
      const float mag = phi(pre[j] + suf);
      const float e = (((sg >> j) ^ tot) & 1u) ? -mag : mag;
      if (store) Et[(e0 + j) * TW + lane] = e;
      suf += ph[j];
    }
  }
  return par;
}

// Variable-node sum (Eq. 7): R_v + sum of the incoming c->v messages in
// ascending check order.  DV as DC above.
template <int DV>
__device__ __forceinline__ float var_sum(const float *__restrict__ Rt, const float *__restrict__ Et,
                                         const int32_t *__restrict__ var_edges, int p0, int dv, int v, int lane) {
  constexpr int DMAX = DV > 0 ? DV : -DV;
  constexpr bool FIXED = DV > 0;
  float ev[DMAX];
#pragma unroll
  for (int j = 0; j < DMAX; ++j)
    if (FIXED || j < dv) ev[j] = Et[var_edges[p0 + j] * TW + lane];
  float s = Rt[v * TW + lane];
#pragma unroll
  for (int j = 0; j < DMAX; ++j)
    if (FIXED || j < dv) s += ev[j];
  return s;
}

}  // namespace ldpc
