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
// (relative error below 1e-6 over [0, inf), below 4e-7 for x < 10):
//   x >= 2 (q = e^-x <= 0.136): the odd series 2 atanh(q) = 2q (1 + q^2/3 + q^4/5 + q^6/7),
//                               truncation < 2e-9;
//   x <  2: phi = log((2 - d) / d) with d = 1 - e^-x, where d comes from the Taylor
//           series x (1 - x/2 + x^2/6 - x^3/24 + x^4/120) for x < 0.15 (no cancellation)
//           and from 1 - q above.
// The check rule applies phi twice with a sum in between, so the inner sum is kept
// in base-2 units (phi / ln 2): phi_to2 takes x and returns phi(x) / ln 2, phi_from2
// takes y = x / ln 2 and returns phi(x).  e^-x = 2^(-x log2 e); the rounding of that
// product only affects phi(x) for large x, where phi is tiny and only enters sums.
constexpr float kL2e = 1.44269504088896341f;  // log2(e) = 1 / ln 2
constexpr float kLn2 = 0.693147180559945309f;

__device__ __forceinline__ float phi_core(float x, float q, float c) {
  // x: argument, q = e^-x; returns c * phi(x) on the series path and the base-2
  // logarithm of (2 - d) / d on the other (the caller scales it)
  const float s = q * q;
  float p = fmaf(s, c / 7.0f, c / 5.0f);
  p = fmaf(s, p, c / 3.0f);
  p = fmaf(s, p, c);
  const float big = q * p;
  float t = fmaf(x, 1.0f / 120.0f, -1.0f / 24.0f);
  t = fmaf(x, t, 1.0f / 6.0f);
  t = fmaf(x, t, -0.5f);
  t = fmaf(x, t, 1.0f);
  const float d = x < 0.15f ? x * t : 1.0f - q;
  const float r = (2.0f - d) * __builtin_amdgcn_rcpf(d);
  const float lg = __builtin_amdgcn_logf(r);
  return x >= 2.0f ? big : lg;
}

// phi(x) / ln 2 for x in [0, inf]
__device__ __forceinline__ float phi_to2(float x) {
  x = fminf(x, 100.0f);  // phi(100) < 1e-43: the result is 0 either way
  const float q = __builtin_amdgcn_exp2f(-x * kL2e);
  return phi_core(x, q, 2.0f * kL2e);
}

// phi(y ln 2) for y in [0, inf]
__device__ __forceinline__ float phi_from2(float y) {
  y = fminf(y, 100.0f * kL2e);
  const float q = __builtin_amdgcn_exp2f(-y);
  const float v = phi_core(y * kLn2, q, 2.0f);
  return y * kLn2 >= 2.0f ? v : v * kLn2;
}

// phi(x) in natural units
__device__ __forceinline__ float phi(float x) { return phi_from2(x * kL2e); }

__device__ __forceinline__ float clamp_msg(float x) { return fminf(fmaxf(x, -kLmax), kLmax); }

// Check rule (Eq. 5) on one lane's incoming messages mv[0..dc) (already clamped):
// E_j = sign_j * phi(sum_{i != j} phi(|M_i|)) with the exclusive sum built from a
// prefix and a suffix (no total-minus-self).  sign_j is the product of the other
// messages' signs, taken from the IEEE sign bits (as the tanh product would give it,
// including the sign of zeros): the XOR of all sign bits with M_j's own.
// DC > 0: degree fixed at compile time; DC < 0: any degree up to -DC (runtime dc).
template <int DC>
__device__ __forceinline__ void check_core(const float *mv, int dc, float *eout) {
  constexpr int DMAX = DC > 0 ? DC : -DC;
  constexpr bool FIXED = DC > 0;
  float ph[DMAX], pre[DMAX];
  uint32_t sx = 0;
#pragma unroll
  for (int j = 0; j < DMAX; ++j) {
    if (FIXED || j < dc) {
      sx ^= __float_as_uint(mv[j]);
      ph[j] = phi_to2(fabsf(mv[j]));  // base-2 units
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
  float suf = 0.0f;
#pragma unroll
  for (int j = DMAX - 1; j >= 0; --j) {
    if (FIXED || j < dc) {
      const float mag = phi_from2(pre[j] + suf);
      const uint32_t sgn = (sx ^ __float_as_uint(mv[j])) & 0x80000000u;
      eout[j] = __uint_as_float(sgn | __float_as_uint(mag));
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
