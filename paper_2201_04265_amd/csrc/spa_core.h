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

// phi(x) = log((e^x + 1) / (e^x - 1)) = 2 atanh(e^-x) for x >= 0: the magnitude map
// of the tanh rule, 2 atanh(prod tanh(a_i / 2)) = phi(sum phi(a_i)).  phi(0) = +inf
// and phi(+inf) = 0, so a zero input message zeroes the others.
// Evaluated from the hardware exp2 / log2 / reciprocal with two branch-free paths
// (relative error a few 1e-7 over [0, inf)):
//   x >= 1.386 (q = e^-x <= 1/4): the odd series 2 atanh(q) = 2q (1 + q^2/3 + ... + q^10/11),
//                                 truncation < 5e-9;
//   x <  1.386: phi = log((2 - d) / d) with d = 1 - e^-x, where d comes from the Taylor
//               series of 1 - e^-x for x < 0.3 (no cancellation) and from 1 - q above.
// e^-x is 2^-(x log2 e) with the product split in two parts, so q keeps ~1 ulp for x <= 20.
__device__ __forceinline__ float phi(float x) {
  constexpr float kL2eHi = 1.44269502162933349609375f;  // log2(e) rounded to float
  constexpr float kL2eLo = 1.925963033500011079e-08f;   // log2(e) - kL2eHi
  constexpr float kLn2 = 0.693147180559945309f;
  x = fminf(x, 100.0f);  // phi(100) < 1e-43: the result is 0 either way, the split stays finite
  const float y = x * kL2eHi;
  const float ey = fmaf(x, kL2eHi, -y) + x * kL2eLo;
  float q = __builtin_amdgcn_exp2f(-y);
  q = fmaf(-q, ey * kLn2, q);  // 2^-(y + ey) ~ 2^-y (1 - ey ln 2)
  const float s = q * q;
  float p = fmaf(s, 1.0f / 11.0f, 1.0f / 9.0f);
  p = fmaf(s, p, 1.0f / 7.0f);
  p = fmaf(s, p, 1.0f / 5.0f);
  p = fmaf(s, p, 1.0f / 3.0f);
  p = fmaf(s, p, 1.0f);
  const float big = 2.0f * q * p;
  float t = fmaf(x, 1.0f / 5040.0f, -1.0f / 720.0f);
  t = fmaf(x, t, 1.0f / 120.0f);
  t = fmaf(x, t, -1.0f / 24.0f);
  t = fmaf(x, t, 1.0f / 6.0f);
  t = fmaf(x, t, -0.5f);
  t = fmaf(x, t, 1.0f);
  const float d = x < 0.3f ? x * t : 1.0f - q;
  const float r = (2.0f - d) * __builtin_amdgcn_rcpf(d);
  const float small = __builtin_amdgcn_logf(r) * kLn2;
  return x >= 1.386f ? big : small;
}

__device__ __forceinline__ float clamp_msg(float x) { return fminf(fmaxf(x, -kLmax), kLmax); }

// Check rule (Eq. 5) on one lane's incoming messages mv[0..dc) (already clamped):
// E_j = sign_j * phi(sum_{i != j} phi(|M_i|)) with the exclusive sum built from a
// prefix and a suffix (no total-minus-self), sign_j = parity of the other signs.
// DC > 0: degree fixed at compile time; DC < 0: any degree up to -DC (runtime dc).
template <int DC>
__device__ __forceinline__ void check_core(const float *mv, int dc, float *eout) {
  constexpr int DMAX = DC > 0 ? DC : -DC;
  constexpr bool FIXED = DC > 0;
  float ph[DMAX], pre[DMAX];
  uint32_t sg = 0;
#pragma unroll
  for (int j = 0; j < DMAX; ++j) {
    if (FIXED || j < dc) {
      sg |= (mv[j] < 0.0f ? 1u : 0u) << j;
      ph[j] = phi(fabsf(mv[j]));
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
      eout[j] = (((sg >> j) ^ tot) & 1u) ? -mag : mag;
      suf += ph[j];
    }
  }
}

// Check-node update of one check for the 64 words of a tile.
//   Mt: v->c messages [nnz][64] (clamped); Et: new c->v messages [nnz][64];
//   Zt: hard-decision masks [n] (bit l = decision of lane l's word).
// Returns the parity of the decisions over the check: the syndrome bit (Eq. 1) of
// the decisions the incoming messages were computed with.
template <int DC>
__device__ __forceinline__ int check_update(const float *__restrict__ Mt, float *__restrict__ Et,
                                            const unsigned long long *Zt, const int32_t *__restrict__ col_idx,
                                            int e0, int dc, int lane, bool store) {
  constexpr int DMAX = DC > 0 ? DC : -DC;
  constexpr bool FIXED = DC > 0;
  float mv[DMAX], ev[DMAX];
  unsigned long long zx = 0;
#pragma unroll
  for (int j = 0; j < DMAX; ++j) {
    if (FIXED || j < dc) {
      mv[j] = Mt[(e0 + j) * TW + lane];
      zx ^= Zt[col_idx[e0 + j]];
    }
  }
  check_core<DC>(mv, dc, ev);
#pragma unroll
  for (int j = 0; j < DMAX; ++j)
    if ((FIXED || j < dc) && store) Et[(e0 + j) * TW + lane] = ev[j];
  return (int)((zx >> lane) & 1ull);
}

// Posterior of one variable (Eq. 7): R_v + the incoming c->v messages in ascending
// check order.  Also returns the running prefixes pre[j] = R_v + sum_{i<j} E_i and
// the messages themselves for the exclusive sums of Eq. 6.  DV as DC above.
template <int DV>
__device__ __forceinline__ float var_posterior(float r, const float *__restrict__ Et,
                                               const int32_t *__restrict__ var_edges, int p0, int dv, int lane,
                                               float *ev, float *pre, int *eid) {
  constexpr int DMAX = DV > 0 ? DV : -DV;
  constexpr bool FIXED = DV > 0;
#pragma unroll
  for (int j = 0; j < DMAX; ++j) {
    if (FIXED || j < dv) {
      eid[j] = var_edges[p0 + j];
      ev[j] = Et[eid[j] * TW + lane];
    }
  }
  float acc = r;
#pragma unroll
  for (int j = 0; j < DMAX; ++j) {
    if (FIXED || j < dv) {
      pre[j] = acc;
      acc += ev[j];
    }
  }
  return acc;
}

// Variable-node update: posterior L (Eq. 7) -> decision mask Zt[v] (Eq. 8, z = [L <= 0]),
// and the v->c messages M_j = clamp(R_v + sum_{i != j} E_i) (Eq. 6) as prefix + suffix.
// With ZERO_E, lanes with `fresh` set see all incoming messages as 0 (a word that has
// not been through a check phase yet): M = clamp(R), z = [R <= 0].
template <int DV, bool ZERO_E = false>
__device__ __forceinline__ void var_update(const float *__restrict__ Rt, const float *__restrict__ Et,
                                           float *__restrict__ Mt, unsigned long long *Zt,
                                           const int32_t *__restrict__ var_edges, int p0, int dv, int v, int lane,
                                           bool store, bool fresh = false) {
  constexpr int DMAX = DV > 0 ? DV : -DV;
  constexpr bool FIXED = DV > 0;
  float ev[DMAX], pre[DMAX];
  int eid[DMAX];
  const float r = Rt[v * TW + lane];
  float L = var_posterior<DV>(r, Et, var_edges, p0, dv, lane, ev, pre, eid);
  if (ZERO_E && fresh) {
#pragma unroll
    for (int j = 0; j < DMAX; ++j) {
      ev[j] = 0.0f;
      pre[j] = r;
    }
    L = r;
  }
  const unsigned long long z = __ballot(L <= 0.0f);
  if (lane == 0) Zt[v] = z;
  float suf = 0.0f;
#pragma unroll
  for (int j = DMAX - 1; j >= 0; --j) {
    if (FIXED || j < dv) {
      if (store) Mt[eid[j] * TW + lane] = clamp_msg(pre[j] + suf);
      suf += ev[j];
    }
  }
}

}  // namespace ldpc
