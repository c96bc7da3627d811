// On-device word generation: systematic GF(2) encoding (Sec. II-A, Eqs. 1-3;
// the systematic generator [I_k : P] of Sec. III-B), BPSK over AWGN (Sec. II-B,
// Eq. 4) with counter-based Philox4x64-10 draws, and decision error counts.
//
// Systematic form.  H is reduced over GF(2) on the host (Gauss-Jordan on
// bit-packed rows), pivot columns chosen from the last column towards the
// first; the non-pivot columns, ascending, carry the k message bits and pivot
// row r fixes bit pivot[r] as the parity of the message bits it touches.  The
// device keeps that map as A [rank][kwp] 64-bit words (bit j of row r = message
// bit j is in the parity of row r) and a column map (message index, or -1 - r).
//
// Encode kernel: one workgroup (4 waves) per tile of 64 words, lane = word.
//   1. the 64 messages are packed to LDS as msg[q][64] (64-bit chunk q of each
//      word), from bytes by ballots or straight from Philox draws;
//   2. each wave takes groups of 4 rows of A: a lane ANDs its message chunk with
//      the 4 rows' chunks (wave-uniform, scalar loads) and accumulates popcounts;
//      a ballot of the low bits gives the 64 words' parity bits of each row
//      (LDS par[r]);
//   3. each wave writes whole codeword rows (and LLRs in the fused form), four
//      consecutive positions per lane.
// GF(2) products of bit-packed operands are 64 multiply-adds per AND + popcount,
// which keeps this on the vector ALU rather than the matrix cores (an int8 MFMA
// would need one byte per bit).
//
// Random draws (Philox4x64-10, Salmon et al., SC 2011):
//   message bits of word w: key (seed, 1), counter (w, j, 0, 0) -> bits
//     256 j .. 256 j + 255, bit i = bit (i mod 64) of output (i div 64) mod 4;
//   noise of word w, positions 4j .. 4j+3: key (seed, 2), counter (w, j, stream, 0)
//     -> (x0, x1, x2, x3); Box-Muller on (x0, x1) gives positions 4j, 4j+1 (cos,
//     sin), on (x2, x3) positions 4j+2, 4j+3, with u1 = (x >> 11 + 1) 2^-53 in
//     (0, 1] and u2 = (x >> 11) 2^-53 in [0, 1).
// LLR lambda = 2 (1 - 2c + sigma z) / sigma^2 in FP64, rounded once for FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace {

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;
constexpr uint64_t kDomainMessage = 1;
constexpr uint64_t kDomainNoise = 2;
constexpr int kEncodeThreads = 256;
constexpr int kRowGroup = 4;
constexpr double kTwoPi = 2.0 * 3.141592653589793;  // the double nearest 2 pi

struct Philox4 {
  uint64_t x0, x1, x2, x3;
};

__device__ inline Philox4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                        uint64_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint64_t hi0 = __umul64hi(kPhiloxM0, c0), lo0 = kPhiloxM0 * c0;
    const uint64_t hi1 = __umul64hi(kPhiloxM1, c2), lo1 = kPhiloxM1 * c2;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
  return {c0, c1, c2, c3};
}

// Two standard normals from two 64-bit draws (Box-Muller).
__device__ inline void box_muller(uint64_t xa, uint64_t xb, double &za, double &zb) {
#pragma clang fp contract(off)
  const double u1 = (double)((xa >> 11) + 1) * 0x1p-53;
  const double u2 = (double)(xb >> 11) * 0x1p-53;
  const double r = sqrt(-2.0 * log(u1));
  const double t = kTwoPi * u2;
  za = r * cos(t);
  zb = r * sin(t);
}

struct ChannelArgs {
  double sigma, sigma2;
  uint64_t seed, stream;
};

// LLRs of positions 4j .. 4j+3 of word w (absolute index) for code bits c[0..3].
__device__ inline void channel_group(const ChannelArgs &ch, uint64_t w, uint64_t j, const uint32_t c[4],
                                     double lam[4]) {
#pragma clang fp contract(off)
  const Philox4 x = philox4x64_10(w, j, ch.stream, 0, ch.seed, kDomainNoise);
  double z[4];
  box_muller(x.x0, x.x1, z[0], z[1]);
  box_muller(x.x2, x.x3, z[2], z[3]);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double xs = 1.0 - 2.0 * (double)c[i];
    const double y = xs + ch.sigma * z[i];
    lam[i] = 2.0 * y / ch.sigma2;
  }
}

template <bool F64>
__device__ inline void store_llr_group(void *llr, size_t row, int n, int v0, const double lam[4], bool full) {
  if (F64) {
    double *o = (double *)llr + row * (size_t)n + v0;
    if (full) {
      *(double2 *)o = make_double2(lam[0], lam[1]);
      *(double2 *)(o + 2) = make_double2(lam[2], lam[3]);
    } else {
      for (int i = 0; i < 4 && v0 + i < n; ++i) o[i] = lam[i];
    }
  } else {
    float *o = (float *)llr + row * (size_t)n + v0;
    if (full) {
      *(float4 *)o = make_float4((float)lam[0], (float)lam[1], (float)lam[2], (float)lam[3]);
    } else {
      for (int i = 0; i < 4 && v0 + i < n; ++i) o[i] = (float)lam[i];
    }
  }
}

struct EncodeDev {
  const uint64_t *A;       // [rank4][kwp]
  const int32_t *colmap;   // [n]
  int32_t n, k, kw, kwp, rank4;
};

// MODE 0: messages from bytes, codewords out.  MODE 1: messages drawn (Philox),
// codewords and LLRs out, messages out if msg_out != nullptr.
template <int MODE, bool F64>
__global__ __launch_bounds__(kEncodeThreads) void encode_kernel(EncodeDev e, const uint8_t *__restrict__ msg_in,
                                                                 int32_t batch, int64_t first_word, ChannelArgs ch,
                                                                 uint8_t *__restrict__ msg_out,
                                                                 uint8_t *__restrict__ cw, void *__restrict__ llr) {
  extern __shared__ __align__(16) uint64_t enc_smem[];
  uint64_t *msg = enc_smem;                        // [kw][64]
  uint64_t *par = enc_smem + (size_t)e.kw * 64;    // [rank4]
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t w0 = (int64_t)blockIdx.x * kTile;
  const int nw = (int)min<int64_t>(kTile, batch - w0);

  // 1. messages -> msg[q][word]
  if constexpr (MODE == 0) {
    for (int w = wid; w < kTile; w += kEncodeThreads / 64) {
      const uint8_t *row = msg_in + (size_t)(w0 + w) * e.k;
      for (int q = 0; q < e.kw; ++q) {
        const int i = q * 64 + lane;
        const bool one = w < nw && i < e.k && row[i] != 0;
        const uint64_t b = __ballot(one);
        if (lane == 0) msg[q * 64 + w] = b;
      }
    }
  } else {
    const int nblk = (e.kw + 3) / 4;
    for (int t = threadIdx.x; t < kTile * nblk; t += kEncodeThreads) {
      const int w = t & 63, j = t >> 6;
      const Philox4 x = philox4x64_10((uint64_t)(first_word + w0 + w), (uint64_t)j, 0, 0, ch.seed, kDomainMessage);
      const uint64_t xs[4] = {x.x0, x.x1, x.x2, x.x3};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int q = 4 * j + i;
        if (q >= e.kw) break;
        const int rem = e.k - 64 * q;
        const uint64_t keep = rem >= 64 ? ~0ull : ((1ull << rem) - 1);
        msg[q * 64 + w] = w < nw ? (xs[i] & keep) : 0ull;
      }
    }
  }
  __syncthreads();

  // 2. parity bits of every row for the 64 words -> par[r]
  for (int r0 = wid * kRowGroup; r0 < e.rank4; r0 += kRowGroup * (kEncodeThreads / 64)) {
    const uint64_t *a0 = e.A + (size_t)r0 * e.kwp;
    const uint64_t *a1 = a0 + e.kwp, *a2 = a1 + e.kwp, *a3 = a2 + e.kwp;
    uint32_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int q = 0; q < e.kw; ++q) {
      const uint64_t m = msg[q * 64 + lane];
      s0 += __popcll(a0[q] & m);
      s1 += __popcll(a1[q] & m);
      s2 += __popcll(a2[q] & m);
      s3 += __popcll(a3[q] & m);
    }
    const uint64_t b0 = __ballot(s0 & 1), b1 = __ballot(s1 & 1), b2 = __ballot(s2 & 1), b3 = __ballot(s3 & 1);
    if (lane == 0) {
      par[r0] = b0;
      par[r0 + 1] = b1;
      par[r0 + 2] = b2;
      par[r0 + 3] = b3;
    }
  }
  __syncthreads();

  // 3. codeword rows (and messages, LLRs)
  const int ngrp = (e.n + 3) / 4;
  const bool n4 = (e.n & 3) == 0;
  for (int w = wid; w < nw; w += kEncodeThreads / 64) {
    const size_t row = (size_t)(w0 + w);
    const uint64_t wbit = 1ull << w;
    for (int g = lane; g < ngrp; g += 64) {
      const int v0 = 4 * g;
      uint32_t c[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int v = v0 + i;
        uint32_t bit = 0;
        if (v < e.n) {
          const int32_t src = e.colmap[v];
          bit = src >= 0 ? (uint32_t)((msg[(src >> 6) * 64 + w] >> (src & 63)) & 1ull)
                         : (uint32_t)((par[-1 - src] & wbit) != 0);
        }
        c[i] = bit;
      }
      uint8_t *o = cw + row * (size_t)e.n + v0;
      if (n4) {
        *(uint32_t *)o = c[0] | (c[1] << 8) | (c[2] << 16) | (c[3] << 24);
      } else {
        for (int i = 0; i < 4 && v0 + i < e.n; ++i) o[i] = (uint8_t)c[i];
      }
      if constexpr (MODE == 1) {
        double lam[4];
        channel_group(ch, (uint64_t)(first_word + (int64_t)row), (uint64_t)g, c, lam);
        store_llr_group<F64>(llr, row, e.n, v0, lam, n4);
      }
    }
    if (MODE == 1 && msg_out != nullptr) {
      uint8_t *mo = msg_out + row * (size_t)e.k;
      for (int i = lane; i < e.k; i += 64) mo[i] = (uint8_t)((msg[(i >> 6) * 64 + w] >> (i & 63)) & 1ull);
    }
  }
}

template <bool F64>
__global__ __launch_bounds__(256) void awgn_kernel(const uint8_t *__restrict__ cw, int32_t n, int64_t groups_total,
                                                   int32_t ngrp, int64_t first_word, ChannelArgs ch,
                                                   void *__restrict__ llr) {
  const bool n4 = (n & 3) == 0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < groups_total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = t / ngrp;
    const int g = (int)(t - row * ngrp);
    const int v0 = 4 * g;
    const uint8_t *in = cw + (size_t)row * n + v0;
    uint32_t c[4];
    if (n4) {
      const uint32_t p = *(const uint32_t *)in;
#pragma unroll
      for (int i = 0; i < 4; ++i) c[i] = ((p >> (8 * i)) & 0xffu) != 0;
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) c[i] = v0 + i < n ? (in[i] != 0) : 0u;
    }
    double lam[4];
    channel_group(ch, (uint64_t)(first_word + row), (uint64_t)g, c, lam);
    store_llr_group<F64>(llr, (size_t)row, n, v0, lam, n4);
  }
}

// counts[0] += decision errors over all positions, counts[1] += over message
// positions, counts[2] += words with at least one error.  One wave per word.
__global__ __launch_bounds__(256) void count_errors_kernel(const uint8_t *__restrict__ hard,
                                                           const uint8_t *__restrict__ cw,
                                                           const int32_t *__restrict__ colmap, int32_t n,
                                                           int32_t batch, bool vec, unsigned long long *counts) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  unsigned long long all = 0, info = 0, words = 0;
  for (int64_t w = wave; w < batch; w += nwaves) {
    const uint8_t *h = hard + (size_t)w * n, *c = cw + (size_t)w * n;
    uint32_t a = 0, b = 0;
    if (vec) {  // rows 4-byte aligned: four positions per lane and load
      for (int v = 4 * lane; v < n; v += 256) {
        const uint32_t hh = *(const uint32_t *)(h + v), cc = *(const uint32_t *)(c + v);
        const int4 cm = *(const int4 *)(colmap + v);
        const int32_t cms[4] = {cm.x, cm.y, cm.z, cm.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t d = (((hh >> (8 * i)) & 0xffu) != 0) != (((cc >> (8 * i)) & 0xffu) != 0);
          a += d;
          b += d & (uint32_t)(cms[i] >= 0);
        }
      }
    } else {
      for (int v = lane; v < n; v += 64) {
        const uint32_t d = (h[v] != 0) != (c[v] != 0);
        a += d;
        b += d & (uint32_t)(colmap[v] >= 0);
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      a += __shfl_xor(a, off);
      b += __shfl_xor(b, off);
    }
    all += a;
    info += b;
    words += a != 0;
  }
  if (lane == 0 && all + info + words) {
    atomicAdd(&counts[0], all);
    atomicAdd(&counts[1], info);
    atomicAdd(&counts[2], words);
  }
}

size_t encode_lds_bytes(const ldpc_encoder_s *e) { return (size_t)e->kw * 64 * 8 + (size_t)e->rank4 * 8; }

EncodeDev encode_dev(const ldpc_encoder_s *e) {
  EncodeDev d;
  d.A = e->d_A;
  d.colmap = e->d_colmap;
  d.n = e->n;
  d.k = e->k;
  d.kw = e->kw;
  d.kwp = e->kwp;
  d.rank4 = e->rank4;
  return d;
}

template <int MODE, bool F64>
ldpc_status launch_encode(const ldpc_encoder_s *e, const uint8_t *msg_in, int32_t batch, int64_t first_word,
                          const ChannelArgs &ch, uint8_t *msg_out, uint8_t *cw, void *llr, hipStream_t stream) {
  const size_t lds = encode_lds_bytes(e);
  if (lds > (size_t)e->lds_limit)
    return set_error(LDPC_ERR_UNSUPPORTED, "encoder state of a 64-word tile (" + std::to_string(lds) +
                                               " bytes) exceeds LDS (" + std::to_string(e->lds_limit) + ")");
  if (batch == 0) return LDPC_OK;
  if (lds > 65536)
    LDPC_HIP_CHECK(hipFuncSetAttribute((const void *)encode_kernel<MODE, F64>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  const unsigned tiles = (unsigned)((batch + kTile - 1) / kTile);
  hipLaunchKernelGGL((encode_kernel<MODE, F64>), dim3(tiles), dim3(kEncodeThreads), lds, stream, encode_dev(e), msg_in, batch,
                     first_word, ch, msg_out, cw, llr);
  LDPC_HIP_CHECK(hipGetLastError());
  return LDPC_OK;
}

}  // namespace

extern "C" ldpc_status ldpc_encoder_create(ldpc_graph_t g, ldpc_encoder_t *out) {
  if (!g || !out) return set_error(LDPC_ERR_INVALID_ARG, "graph or out is NULL");
  *out = nullptr;
  std::vector<int32_t> pivots;
  std::vector<uint64_t> rows;
  int W = 0;
  systematic_form(g, pivots, rows, W);
  ldpc_encoder_s *e = new (std::nothrow) ldpc_encoder_s();
  if (!e) return set_error(LDPC_ERR_OUT_OF_MEMORY, "encoder allocation");
  const int n = g->n, rank = (int)pivots.size();
  e->n = n;
  e->rank = rank;
  e->k = n - rank;
  e->kw = (e->k + 63) / 64;
  e->kwp = std::max(1, e->kw);
  e->rank4 = (rank + kRowGroup - 1) / kRowGroup * kRowGroup;
  e->pivots = pivots;
  std::vector<int32_t> colmap(n, 0);
  std::vector<char> is_pivot(n, 0);
  for (int r = 0; r < rank; ++r) {
    is_pivot[pivots[r]] = 1;
    colmap[pivots[r]] = -1 - r;
  }
  for (int v = 0; v < n; ++v)
    if (!is_pivot[v]) {
      colmap[v] = (int32_t)e->info.size();
      e->info.push_back(v);
    }
  std::vector<uint64_t> A((size_t)e->rank4 * e->kwp, 0);
  for (int r = 0; r < rank; ++r)
    for (int j = 0; j < e->k; ++j) {
      const int v = e->info[j];
      if (rows[(size_t)r * W + (v >> 6)] >> (v & 63) & 1ull) A[(size_t)r * e->kwp + (j >> 6)] |= 1ull << (j & 63);
    }
  int dev = 0, lim = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err == hipSuccess) err = hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (err == hipSuccess) err = hipMalloc((void **)&e->d_A, A.size() * sizeof(uint64_t));
  if (err == hipSuccess) err = hipMalloc((void **)&e->d_colmap, (size_t)n * sizeof(int32_t));
  if (err == hipSuccess) err = hipMemcpy(e->d_A, A.data(), A.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
  if (err == hipSuccess)
    err = hipMemcpy(e->d_colmap, colmap.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice);
  if (err != hipSuccess) {
    if (e->d_A) (void)hipFree(e->d_A);
    if (e->d_colmap) (void)hipFree(e->d_colmap);
    delete e;
    return hip_error(err, "encoder device arrays");
  }
  e->device = dev;
  e->lds_limit = lim;
  *out = e;
  return LDPC_OK;
}

extern "C" ldpc_status ldpc_encoder_destroy(ldpc_encoder_t e) {
  if (!e) return set_error(LDPC_ERR_INVALID_ARG, "encoder is NULL");
  if (e->d_A) (void)hipFree(e->d_A);
  if (e->d_colmap) (void)hipFree(e->d_colmap);
  delete e;
  return LDPC_OK;
}

extern "C" ldpc_status ldpc_encoder_info(ldpc_encoder_t e, int32_t *n, int32_t *k, int32_t *rank) {
  if (!e) return set_error(LDPC_ERR_INVALID_ARG, "encoder is NULL");
  if (n) *n = e->n;
  if (k) *k = e->k;
  if (rank) *rank = e->rank;
  return LDPC_OK;
}

extern "C" ldpc_status ldpc_encoder_positions(ldpc_encoder_t e, int32_t *info, int32_t *pivots) {
  if (!e) return set_error(LDPC_ERR_INVALID_ARG, "encoder is NULL");
  if (info && e->k) std::memcpy(info, e->info.data(), (size_t)e->k * sizeof(int32_t));
  if (pivots && e->rank) std::memcpy(pivots, e->pivots.data(), (size_t)e->rank * sizeof(int32_t));
  return LDPC_OK;
}

extern "C" ldpc_status ldpc_encode(ldpc_encoder_t e, const uint8_t *msg, int32_t batch, uint8_t *cw,
                                   hipStream_t stream) {
  if (!e) return set_error(LDPC_ERR_INVALID_ARG, "encoder is NULL");
  if (batch < 0) return set_error(LDPC_ERR_INVALID_ARG, "batch < 0");
  if (batch > 0 && (!cw || (e->k > 0 && !msg))) return set_error(LDPC_ERR_INVALID_ARG, "NULL buffer");
  if ((uintptr_t)cw & 3) return set_error(LDPC_ERR_INVALID_ARG, "cw must be 4-byte aligned");
  ChannelArgs ch{};
  return launch_encode<0, false>(e, msg, batch, 0, ch, nullptr, cw, nullptr, stream);
}

namespace {
ldpc_status channel_args(double sigma2, uint64_t seed, uint64_t noise_stream, int64_t first_word, int32_t batch,
                         uint32_t flags, ChannelArgs &ch) {
  if (!(sigma2 > 0.0) || !std::isfinite(sigma2)) return set_error(LDPC_ERR_INVALID_ARG, "sigma2 must be > 0");
  if (first_word < 0 || first_word > INT64_MAX - batch) return set_error(LDPC_ERR_INVALID_ARG, "first_word out of range");
  if (flags & ~LDPC_LLR_F64) return set_error(LDPC_ERR_INVALID_ARG, "unknown flag");
  ch.sigma2 = sigma2;
  ch.sigma = std::sqrt(sigma2);
  ch.seed = seed;
  ch.stream = noise_stream;
  return LDPC_OK;
}
}  // namespace

extern "C" ldpc_status ldpc_channel_awgn(const uint8_t *cw, int32_t batch, int32_t n, double sigma2, uint64_t seed,
                                         uint64_t noise_stream, int64_t first_word, uint32_t flags, void *llr,
                                         hipStream_t stream) {
  if (batch < 0 || n <= 0) return set_error(LDPC_ERR_INVALID_ARG, "batch < 0 or n <= 0");
  ChannelArgs ch{};
  ldpc_status st = channel_args(sigma2, seed, noise_stream, first_word, batch, flags, ch);
  if (st != LDPC_OK) return st;
  if (batch == 0) return LDPC_OK;
  if (!cw || !llr) return set_error(LDPC_ERR_INVALID_ARG, "NULL buffer");
  if (((uintptr_t)cw & 3) || ((uintptr_t)llr & 15)) return set_error(LDPC_ERR_INVALID_ARG, "misaligned buffer");
  const int32_t ngrp = (n + 3) / 4;
  const int64_t total = (int64_t)batch * ngrp;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 1 << 20);
  if (flags & LDPC_LLR_F64)
    hipLaunchKernelGGL(awgn_kernel<true>, dim3(blocks), dim3(256), 0, stream, cw, n, total, ngrp, first_word, ch,
                       llr);
  else
    hipLaunchKernelGGL(awgn_kernel<false>, dim3(blocks), dim3(256), 0, stream, cw, n, total, ngrp, first_word, ch,
                       llr);
  LDPC_HIP_CHECK(hipGetLastError());
  return LDPC_OK;
}

extern "C" ldpc_status ldpc_generate(ldpc_encoder_t e, int32_t batch, uint64_t seed, uint64_t noise_stream,
                                     int64_t first_word, double sigma2, uint32_t flags, uint8_t *msg, uint8_t *cw,
                                     void *llr, hipStream_t stream) {
  if (!e) return set_error(LDPC_ERR_INVALID_ARG, "encoder is NULL");
  if (batch < 0) return set_error(LDPC_ERR_INVALID_ARG, "batch < 0");
  ChannelArgs ch{};
  ldpc_status st = channel_args(sigma2, seed, noise_stream, first_word, batch, flags, ch);
  if (st != LDPC_OK) return st;
  if (batch > 0 && (!cw || !llr)) return set_error(LDPC_ERR_INVALID_ARG, "NULL buffer");
  if (((uintptr_t)cw & 3) || ((uintptr_t)llr & 15)) return set_error(LDPC_ERR_INVALID_ARG, "misaligned buffer");
  if (flags & LDPC_LLR_F64) return launch_encode<1, true>(e, nullptr, batch, first_word, ch, msg, cw, llr, stream);
  return launch_encode<1, false>(e, nullptr, batch, first_word, ch, msg, cw, llr, stream);
}

extern "C" ldpc_status ldpc_count_errors(ldpc_encoder_t e, const uint8_t *hard, const uint8_t *cw, int32_t batch,
                                         uint64_t *counts, hipStream_t stream) {
  if (!e) return set_error(LDPC_ERR_INVALID_ARG, "encoder is NULL");
  if (batch < 0) return set_error(LDPC_ERR_INVALID_ARG, "batch < 0");
  if (!counts) return set_error(LDPC_ERR_INVALID_ARG, "counts is NULL");
  if ((uintptr_t)counts & 7) return set_error(LDPC_ERR_INVALID_ARG, "counts must be 8-byte aligned");
  if (batch == 0) return LDPC_OK;
  if (!hard || !cw) return set_error(LDPC_ERR_INVALID_ARG, "NULL buffer");
  const unsigned blocks = (unsigned)std::min<int64_t>(((int64_t)batch + 3) / 4, 2048);
  const bool vec = (e->n & 3) == 0 && ((uintptr_t)hard & 3) == 0 && ((uintptr_t)cw & 3) == 0;
  hipLaunchKernelGGL(count_errors_kernel, dim3(blocks), dim3(256), 0, stream, hard, cw, e->d_colmap, e->n, batch, vec,
                     (unsigned long long *)counts);
  LDPC_HIP_CHECK(hipGetLastError());
  return LDPC_OK;
}
