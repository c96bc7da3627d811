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

// Graph tables (CSR offsets, edge numbering) never change while a decode runs.  Their
// loads go through the constant address space, so an index the whole wavefront shares is
// fetched with a scalar load whatever else the kernel stores to global memory (through a
// plain pointer the compiler must assume those stores may clobber it, and falls back to
// a vector load per wavefront).
template <class T>
__device__ __forceinline__ T ld_graph(const T *p, size_t i) {
  return ((const __attribute__((address_space(4))) T *)p)[i];
}

// Workgroup barrier that orders LDS only: global loads and stores in flight are not
// waited for.  For kernels whose threads exchange data only through LDS (what they
// write to global memory is read by later launches or by the writing thread itself).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

constexpr float kL2e = 1.44269504088896341f;  // log2(e) = 1 / ln 2
constexpr float kLn2 = 0.693147180559945309f;

__device__ __forceinline__ float clamp_msg(float x) { return fminf(fmaxf(x, -kLmax), kLmax); }

// Hard decisions travel with the messages.  A v->c message M (Eq. 6, |M| <= 20) is
// stored as M / 16: exact (a power of two), and |M / 16| <= 1.25 < 2 keeps the top
// exponent bit (bit 30) at 0, so that bit carries the sending variable's decision
// z_v = [L_v <= 0] (Eq. 8) without changing the message's value.  A check reads its
// variables' decisions together with their messages, and its syndrome bit (Eq. 1) is
// the XOR of those bits: no decision arrays and no extra loads.  The check rule takes
// the stored form directly (the 1/16 folds into its first multiply).
constexpr float kMsgDown = 0.0625f;
constexpr uint32_t kDecisionBit = 1u << 30;

// Stored v->c message from the pre-clamp value x, carrying decision z.
__device__ __forceinline__ float v2c_store(float x, bool z) {
  return __uint_as_float(__float_as_uint(clamp_msg(x) * kMsgDown) | (z ? kDecisionBit : 0u));
}

// Check rule (Eq. 5) on one lane's incoming messages mv[0..dc) (already clamped):
// E_j = sign_j * 2 atanh(prod_{i != j} tanh(|M_i| / 2)).
//
// Magnitudes.  With q_i = e^-|M_i|, tanh(|M_i| / 2) = (1 - q_i) / (1 + q_i), so a
// product over a set of messages is B / A with A = prod (1 + q_i), B = prod (1 - q_i),
// and 2 atanh(B / A) = ln((A + B) / (A - B)).  Each set is carried as the pair
// d = (A - B) / 2, s = (A + B) / 2, which only ever adds non-negative terms:
//   one message       (d, s) = (q, 1)            the empty set (0, 1)
//   joining two sets  (d, s) = (d1 s2 + s1 d2, s1 s2 + d1 d2)
// so neither a tanh near 1 (large |M|, where 1 - tanh cancels) nor one near 0 loses
// the difference A - B, and the magnitude is ln(s / d).  The pair of the other messages
// of edge j joins a prefix pair (messages before j) and a suffix pair (after j).
// |M_i| <= 20 keeps q_i >= 2e-9 and d > 0; a zero message (q = 1) gives d = s and so a
// zero output on the others.
//
// Precision (each step chosen so that a stored FP32 message carries about the error of
// its own rounding, which loopy decoding otherwise amplifies along long trajectories):
//  * q: the exponent |M| log2(e) is split into yh (its FP32 rounding) and the residual
//    yl (exact from an fma, plus the constant's low part), and q = 2^-yh (1 - yl ln 2);
//    FP32, within the hardware exp2's error (0.8 ulp) of e^-|M|.
//  * joins: the running pairs accumulate in FP64 (full-rate FMA on this chip), so a
//    chain of joins adds no FP32 rounding.  Only the ratio of a pair matters, so a prefix
//    pair is kept as one FP32 value, tau = d / s (the pair scaled to s = 1), and the
//    pair of the others of edge j is (d_suf + tau s_suf, s_suf + tau d_suf).
//  * output: the ratio s / d in FP64 (the hardware FP64 reciprocal refined by one
//    Newton step), then rounded once to FP32 for the hardware log2.
// Signs.  sign_j is the product of the other messages' signs, taken from the IEEE sign
// bits (as the tanh product would give it, including the sign of zeros): the XOR of
// all sign bits with M_j's own.
// STORED: mv holds stored messages (M / 16 with a decision in bit 30, see v2c_store);
// otherwise plain values M.  Both give the same outputs bit for bit: the exponent is
// formed from |M| / 16 in both cases (exact), times 16 log2(e).  Returns the XOR of the
// input bit patterns: bit 31 is the sign of the product of all messages, and for stored
// messages bit 30 is the parity of the decisions they carry (syndrome_bit).
// DC > 0: degree fixed at compile time; DC < 0: any degree up to -DC (runtime dc).
// AUX: also returns, per edge, q_j = e^-|M_j| in aq and r_j = e^|E_j| (the ratio s / d
// whose logarithm is the output magnitude) in ar, for the adjoint.
// emit(j, E_j) receives the outputs, last edge first, after every input has been read.
constexpr float kYHi = 23.083120346069336f;     // 16 log2(e) rounded to FP32
constexpr float kYLo = 3.0815408536000177e-07f; // 16 log2(e) - kYHi

// q = e^-|M| from x16 = |M| / 16.
__device__ __forceinline__ float msg_q(float x16) {
  const float yh = x16 * kYHi;
  const float yl = fmaf(x16, kYLo, fmaf(x16, kYHi, -yh));
  const float qh = __builtin_amdgcn_exp2f(-yh);
  return fmaf(qh, -yl * kLn2, qh);
}

// b / a for a > 0 in FP64: hardware reciprocal (~5e-8) and one Newton step.
__device__ __forceinline__ double quot64(double b, double a) {
  const double r0 = __builtin_amdgcn_rcp(a);
  const double e = fma(-a, r0, 1.0);
  const double q0 = b * r0;
  return fma(q0, e, q0);
}

// Magnitude ln(ratio) of an output; ratio >= 1 up to rounding (|log2| keeps it >= 0).
__device__ __forceinline__ float ratio_log(double ratio, float &rf) {
  rf = (float)ratio;
  return fabsf(__builtin_amdgcn_logf(rf)) * kLn2;
}

// Prefix pair (d, s) of messages 0..j-1 scaled to s = 1, j >= 1: a single message is
// (q_0, 1) itself; later ones d / s, rounded to FP32.
__device__ __forceinline__ float prefix_tau(int j, float q0, double d, double s) {
  return j == 1 ? q0 : (float)quot64(d, s);
}

// TS > 0: the prefix taus go to tsl[j * TS] (a lane's column of LDS) instead of a register
// array, for high degrees in kernels whose registers are short (same values).
template <int DC, bool STORED = false, bool AUX = false, int TS = 0, class Emit>
__device__ __forceinline__ uint32_t check_core_emit(const float *mv, int dc, Emit emit, float *aq = nullptr,
                                                    float *ar = nullptr, float *tsl = nullptr) {
  constexpr int DMAX = DC > 0 ? DC : -DC;
  constexpr bool FIXED = DC > 0;
  // qs[j] = q_j, and the sign of M_j: for degrees up to 16 the message's bit pattern is
  // kept (mb); above, the sign bit rides in qs[j] so that the messages need not stay live.
  constexpr bool KEEP_BITS = FIXED && DMAX <= 16;
  float qs[DMAX], tr[TS ? 1 : DMAX];  // tr: the prefix taus
  uint32_t mb[KEEP_BITS ? DMAX : 1];
  uint32_t sx = 0;
#pragma unroll
  for (int j = 0; j < DMAX; ++j) {
    if (FIXED || j < dc) {
      const uint32_t b = __float_as_uint(mv[j]);
      sx ^= b;
      const float q = msg_q(STORED ? __uint_as_float(b & 0x3fffffffu) : fabsf(mv[j]) * kMsgDown);
      if (KEEP_BITS) {
        mb[KEEP_BITS ? j : 0] = b;
        qs[j] = q;
      } else {
        qs[j] = __uint_as_float(__float_as_uint(q) | (b & 0x80000000u));
      }
    }
  }
  // Joins with the empty set (0, 1) are written out: they are exact, and 0 * x cannot
  // be folded by the compiler.  A generic degree's last suffix step keeps the general
  // form, which gives the same values.  A suffix pair's s that is the constant 1 in one
  // instantiation and a computed 1.0 in another only ever meets the form fma(tau, s, d),
  // where folding x * 1 leaves one rounding of tau + d either way, so fixed and generic
  // degrees agree bit for bit.
  double d = 0.0, s = 1.0;
#pragma unroll
  for (int j = 0; j < DMAX; ++j) {
    if (FIXED || j < dc) {
      if (j > 0) {  // j = 0: the empty prefix, never read
        const float t = prefix_tau(j, fabsf(qs[0]), d, s);
        if constexpr (TS > 0)
          tsl[j * TS] = t;
        else
          tr[j] = t;
      }
      const double q = (double)fabsf(qs[j]);
      if (j == 0) {
        d = q;
        s = 1.0;
      } else {
        const double dn = fma(s, q, d);
        s = fma(d, q, s);
        d = dn;
      }
    }
  }
  d = 0.0;
  s = 1.0;
#pragma unroll
  for (int j = DMAX - 1; j >= 0; --j) {
    if (FIXED || j < dc) {
      const bool top = FIXED && j == DMAX - 1;  // empty suffix
      double od, os;
      if (j == 0) {
        od = d;
        os = s;
      } else {
        const double t = (double)(TS > 0 ? tsl[j * TS] : tr[TS > 0 ? 0 : j]);
        if (top) {
          od = t;
          os = 1.0;
        } else {
          od = fma(t, s, d);
          os = fma(t, d, s);
        }
      }
      float rf;
      const float mag = ratio_log(quot64(os, od), rf);
      if (AUX) {
        aq[j] = fabsf(qs[j]);
        ar[j] = fmaxf(rf, 1.0f);
      }
      const uint32_t sgn = (sx ^ (KEEP_BITS ? mb[KEEP_BITS ? j : 0] : __float_as_uint(qs[j]))) & 0x80000000u;
      emit(j, __uint_as_float(sgn | __float_as_uint(mag)));
      const double q = (double)fabsf(qs[j]);
      if (top) {
        d = q;
        s = 1.0;
      } else {
        const double dn = fma(s, q, d);
        s = fma(d, q, s);
        d = dn;
      }
    }
  }
  return sx;
}

// The same with the outputs in an array.
template <int DC, bool STORED = false, bool AUX = false>
__device__ __forceinline__ uint32_t check_core(const float *mv, int dc, float *eout, float *aq = nullptr,
                                               float *ar = nullptr) {
  return check_core_emit<DC, STORED, AUX>(mv, dc, [&](int j, float v) { eout[j] = v; }, aq, ar);
}

// check_core for a runtime degree (DC < 0) on stored messages, in place on the check's
// own LDS row: the row holds the inputs, then (while the prefix pairs are formed) the
// prefix taus, then the outputs.  Each row entry is read back before it is overwritten by
// the same thread.  The arithmetic and its order are those of check_core<DC, true>, so
// the outputs are the same bit for bit; the row stands in for the register array of
// prefix taus.  Entry j of the row is row[j * STRIDE] (64 when the 64 checks of a
// wavefront interleave their rows).
template <int DC, int STRIDE = 1>
__device__ __forceinline__ uint32_t check_core_row(float *row, int dc) {
  static_assert(DC < 0, "runtime degrees only");
  constexpr int DMAX = -DC;
  float qs[DMAX];
  uint32_t sx = 0;
#pragma unroll
  for (int j = 0; j < DMAX; ++j) {
    if (j < dc) {
      const uint32_t b = __float_as_uint(row[j * STRIDE]);
      sx ^= b;
      const float q = msg_q(__uint_as_float(b & 0x3fffffffu));
      qs[j] = __uint_as_float(__float_as_uint(q) | (b & 0x80000000u));
    }
  }
  double d = 0.0, s = 1.0;
#pragma unroll
  for (int j = 0; j < DMAX; ++j) {
    if (j < dc) {
      if (j > 0) row[j * STRIDE] = prefix_tau(j, fabsf(qs[0]), d, s);
      const double q = (double)fabsf(qs[j]);
      if (j == 0) {
        d = q;
        s = 1.0;
      } else {
        const double dn = fma(s, q, d);
        s = fma(d, q, s);
        d = dn;
      }
      // one entry at a time: interleaving the unrolled entries would keep their FP64
      // temporaries live together and push high degrees out of registers
      if constexpr (DMAX > 8) __builtin_amdgcn_sched_barrier(0);
    }
  }
  d = 0.0;
  s = 1.0;
#pragma unroll
  for (int j = DMAX - 1; j >= 0; --j) {
    if (j < dc) {
      double od, os;
      if (j == 0) {
        od = d;
        os = s;
      } else {
        const double t = (double)row[j * STRIDE];
        od = fma(t, s, d);
        os = fma(t, d, s);
      }
      float rf;
      const float mag = ratio_log(quot64(os, od), rf);
      const uint32_t sgn = (sx ^ __float_as_uint(qs[j])) & 0x80000000u;
      row[j * STRIDE] = __uint_as_float(sgn | __float_as_uint(mag));
      const double q = (double)fabsf(qs[j]);
      const double dn = fma(s, q, d);
      s = fma(d, q, s);
      d = dn;
      if constexpr (DMAX > 8) __builtin_amdgcn_sched_barrier(0);
    }
  }
  return sx;
}

// check_core_row for a degree that is the same across the wavefront: a switch to the
// instance compiled for that exact degree, whose degree tests all fold away (the
// arithmetic is the same source, so the same bits as the runtime-degree form).
template <int DC, int STRIDE>
__device__ __forceinline__ uint32_t check_core_row_uniform(float *row, int dcu) {
  static_assert(DC < 0, "runtime degrees only");
  uint32_t sx = 0;
  switch (dcu) {
#define LDPC_ROW_CASE(D)                                               \
  case D:                                                              \
    if constexpr (D <= -DC) sx = check_core_row<-D, STRIDE>(row, D); \
    break;
    LDPC_ROW_CASE(2) LDPC_ROW_CASE(3) LDPC_ROW_CASE(4) LDPC_ROW_CASE(5) LDPC_ROW_CASE(6) LDPC_ROW_CASE(7)
    LDPC_ROW_CASE(8) LDPC_ROW_CASE(9) LDPC_ROW_CASE(10) LDPC_ROW_CASE(11) LDPC_ROW_CASE(12) LDPC_ROW_CASE(13)
    LDPC_ROW_CASE(14) LDPC_ROW_CASE(15) LDPC_ROW_CASE(16) LDPC_ROW_CASE(17) LDPC_ROW_CASE(18) LDPC_ROW_CASE(19)
    LDPC_ROW_CASE(20) LDPC_ROW_CASE(21) LDPC_ROW_CASE(22) LDPC_ROW_CASE(23) LDPC_ROW_CASE(24) LDPC_ROW_CASE(25)
    LDPC_ROW_CASE(26) LDPC_ROW_CASE(27) LDPC_ROW_CASE(28) LDPC_ROW_CASE(29) LDPC_ROW_CASE(30) LDPC_ROW_CASE(31)
    LDPC_ROW_CASE(32)
#undef LDPC_ROW_CASE
    default:
      break;
  }
  return sx;
}

// Syndrome bit of a check from the value check_core returned for stored messages.
__device__ __forceinline__ int syndrome_bit(uint32_t sx) { return (int)((sx >> 30) & 1u); }

// Check-node update of one check for the 64 words of a tile.
//   Mt: stored v->c messages [nnz][64] (v2c_store); Et: new c->v messages.
// Returns the parity of the decisions over the check: the syndrome bit (Eq. 1) of
// the decisions the incoming messages were sent with.
template <int DC, int TS = 0>
__device__ __forceinline__ int check_update_core(const float *__restrict__ Mt, float *__restrict__ Et, int e0, int dc,
                                                 int lane, bool store, float *psl) {
  constexpr int DMAX = DC > 0 ? DC : -DC;
  constexpr bool FIXED = DC > 0;
  float mv[DMAX];
#pragma unroll
  for (int j = 0; j < DMAX; ++j)
    if (FIXED || j < dc) mv[j] = Mt[(e0 + j) * TW + lane];
  // outputs go straight to Et (every input has been read by then): no output array
  const uint32_t sx = check_core_emit<DC, true, false, TS>(
      mv, dc, [&](int j, float v) {
        if (store) Et[(e0 + j) * TW + lane] = v;
      },
      nullptr, nullptr, psl);
  return syndrome_bit(sx);
}

// Degrees above this keep the prefix taus in LDS (check_update's psl).
constexpr int kPslDegree = 8;

// LDS floats per wavefront that check_update needs for runtime degrees up to -DC.
template <int DC>
constexpr int check_psl_floats() {
  return (DC > kPslDegree || -DC > kPslDegree) ? (DC > 0 ? DC : -DC) * TW : 0;
}

// Degrees above kPslDegree keep their prefix taus in the wavefront's LDS block psl
// ([|DC|][64] floats; this lane's column), which leaves the high-degree kernels one register
// array of the degree (same values, so the same outputs).
template <int DC>
__device__ __forceinline__ int check_update(const float *__restrict__ Mt, float *__restrict__ Et, int e0, int dc,
                                            int lane, bool store, float *psl = nullptr) {
  if constexpr (check_psl_floats<DC>() > 0)
    return check_update_core<DC, TW>(Mt, Et, e0, dc, lane, store, psl + lane);
  else
    return check_update_core<DC>(Mt, Et, e0, dc, lane, store, nullptr);
}

// Variable-node sums (Eqs. 6-7) in FP64: the posterior L = R_v + sum_i x_i (ascending
// check order) and the extrinsic sums L - x_j, each rounded once to FP32 where it is
// stored.  In FP64 the total-minus-own form loses nothing at FP32 output precision (its
// error is ~1e-16 |L|), and one rounding per stored value instead of a chain of FP32
// additions keeps the per-iteration error near that of correct rounding.  DV as DC above;
// every form of the decoder uses these two functions.
template <int DV>
__device__ __forceinline__ double var_total(float r, const float *x, int dv) {
  constexpr int DMAX = DV > 0 ? DV : -DV;
  double L = (double)r;
#pragma unroll
  for (int j = 0; j < DMAX; ++j)
    if (DV > 0 || j < dv) L += (double)x[j];
  return L;
}

// Extrinsic sum of message j from the FP64 total, rounded once (pre-clamp).
__device__ __forceinline__ float var_extrinsic(double L, float xj) { return (float)(L - (double)xj); }

// Posterior of one variable (Eq. 7), FP64, from the incoming c->v messages of tile
// buffer Et; also returns the messages and their edge ids.  DV as DC above.
template <int DV>
__device__ __forceinline__ double var_posterior(float r, const float *__restrict__ Et,
                                                const int32_t *__restrict__ var_edges, int p0, int dv, int lane,
                                                float *ev, int *eid) {
  constexpr int DMAX = DV > 0 ? DV : -DV;
  constexpr bool FIXED = DV > 0;
#pragma unroll
  for (int j = 0; j < DMAX; ++j) {
    if (FIXED || j < dv) {
      eid[j] = ld_graph(var_edges, p0 + j);
      ev[j] = Et[eid[j] * TW + lane];
    }
  }
  return var_total<DV>(r, ev, dv);
}

// Variable-node update: posterior L (Eq. 7), its decision z = [L <= 0] (Eq. 8, on the
// FP32 posterior), and the v->c messages M_j = clamp(R_v + sum_{i != j} E_i) (Eq. 6),
// stored carrying z.  With ZERO_E, lanes with `fresh` set see all incoming messages as 0
// (a word that has not been through a check phase yet): M = clamp(R), z = [R <= 0].
template <int DV, bool ZERO_E = false>
__device__ __forceinline__ void var_update(const float *__restrict__ Rt, const float *__restrict__ Et,
                                           float *__restrict__ Mt, const int32_t *__restrict__ var_edges, int p0,
                                           int dv, int v, int lane, bool store, bool fresh = false) {
  constexpr int DMAX = DV > 0 ? DV : -DV;
  float ev[DMAX];
  int eid[DMAX];
  const float r = Rt[v * TW + lane];
  double L = var_posterior<DV>(r, Et, var_edges, p0, dv, lane, ev, eid);
  if (ZERO_E && fresh) {
#pragma unroll
    for (int j = 0; j < DMAX; ++j) ev[j] = 0.0f;
    L = (double)r;
  }
  const bool z = (float)L <= 0.0f;
  if (store) {
#pragma unroll
    for (int j = 0; j < DMAX; ++j)
      if (DV > 0 || j < dv) Mt[eid[j] * TW + lane] = v2c_store(var_extrinsic(L, ev[j]), z);
  }
}

}  // namespace ldpc
