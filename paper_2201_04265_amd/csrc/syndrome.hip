// Syndrome test of Eq. 1 on given hard decisions: ok[b] = 1 iff every check of H
// sees an even number of ones among word b's decisions (H z_b^T = 0 over GF(2)).
//
// The decoders apply this test inside their iterations to stop a word early; this
// entry point applies it to any batch of decisions (a decoder's output after a run
// without early stop, or words from elsewhere), so that a caller can tell a word that
// satisfies every check at the iteration limit from one that does not.
//
// Codes of up to kSynPackedMaxN variables: a workgroup takes 32 consecutive
// words at a time.  Their decisions are transposed into LDS as one 32-bit mask per
// variable (bit w = word w's decision; coalesced reads of each row, four decisions per
// load when the rows are 4-byte aligned), then each
// thread takes checks c = tid, tid + 256, ... and XORs the masks of the check's
// variables: 32 syndromes per gather, so the graph's index arrays are read once per 32
// words instead of once per word (for a (3,6) code they are 14 times the decisions'
// bytes).  The threads' unsatisfied-word masks are ORed in LDS.
// Longer codes: one workgroup per word; its decisions are copied to LDS when they fit
// (kSynLdsMax bytes) and gathered from global memory otherwise, and a thread stops at
// its first unsatisfied check.
#include <algorithm>

#include "internal.h"

namespace ldpc {
namespace {

constexpr int kSynThreads = 256;
constexpr int kSynLdsMax = 65536;      // bytes of LDS a workgroup may use without opt-in
constexpr int kSynMaxGrid = 256 * 32;  // workgroups per launch (words beyond are strided)

constexpr int kSynWords = 32;                  // words per group in the packed form
constexpr int kSynPackedMaxN = 32768;          // one 32-bit mask per variable: at most 128 KB of LDS

// Bit 7 of each byte of the result is set iff that byte of x is nonzero.
__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t x) {
  return (((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) | x) & 0x80808080u;
}

// VEC: n % 4 == 0 and a 4-byte aligned batch, so each thread reads four decisions of a
// row with one load.
template <bool VEC>
__global__ void __launch_bounds__(kSynThreads)
    syndrome_packed_kernel(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx, int m, int n,
                           const uint8_t *__restrict__ hard, int batch, uint8_t *__restrict__ ok) {
  extern __shared__ __align__(16) uint32_t zb[];
  __shared__ uint32_t s_unsat[2];  // by group parity: cleared two groups after its last read
  const int groups = batch / kSynWords + (batch % kSynWords != 0);  // no overflow near INT32_MAX
  int parity = 0;
  for (int grp = blockIdx.x; grp < groups; grp += gridDim.x, parity ^= 1) {
    const int b0 = grp * kSynWords;
    const int nw = min(kSynWords, batch - b0);
    if (threadIdx.x == 0) s_unsat[parity] = 0u;
    const uint8_t *z = hard + (size_t)b0 * (size_t)n;
    if constexpr (VEC) {
      const int n4 = n >> 2;
      for (int i = threadIdx.x; i < n4; i += kSynThreads) {
        uint32_t m0 = 0u, m1 = 0u, m2 = 0u, m3 = 0u;
        for (int w = 0; w < nw; ++w) {
          const uint32_t t = nonzero_bytes(((const uint32_t *)(z + (size_t)w * (size_t)n))[i]);
          m0 |= ((t >> 7) & 1u) << w;
          m1 |= ((t >> 15) & 1u) << w;
          m2 |= ((t >> 23) & 1u) << w;
          m3 |= (t >> 31) << w;
        }
        ((uint4 *)zb)[i] = make_uint4(m0, m1, m2, m3);
      }
    } else {
      for (int v = threadIdx.x; v < n; v += kSynThreads) {
        uint32_t mask = 0u;
        for (int w = 0; w < nw; ++w) mask |= (uint32_t)(z[(size_t)w * (size_t)n + v] != 0) << w;
        zb[v] = mask;
      }
    }
    __syncthreads();
    const uint32_t all = nw == kSynWords ? ~0u : (1u << nw) - 1u;
    uint32_t unsat = 0u;
    for (int c = threadIdx.x; c < m && unsat != all; c += kSynThreads) {
      const int e1 = row_ptr[c + 1];
      uint32_t p = 0u;
      for (int e = row_ptr[c]; e < e1; ++e) p ^= zb[col_idx[e]];
      unsat |= p;
    }
    if (unsat) atomicOr(&s_unsat[parity], unsat);
    __syncthreads();  // all gathers and ORs of this group done: zb may be overwritten next
    if (threadIdx.x < nw) ok[b0 + threadIdx.x] = (s_unsat[parity] >> threadIdx.x) & 1u ? 0 : 1;
  }
}

template <bool STAGE>
__global__ void __launch_bounds__(kSynThreads)
    syndrome_kernel(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx, int m, int n,
                    const uint8_t *__restrict__ hard, int batch, uint8_t *__restrict__ ok) {
  extern __shared__ __align__(16) uint8_t zs[];
  for (int b = blockIdx.x; b < batch; b += gridDim.x) {
    const uint8_t *z = hard + (size_t)b * (size_t)n;
    if constexpr (STAGE) {
      for (int v = threadIdx.x; v < n; v += kSynThreads) zs[v] = z[v] != 0;
      __syncthreads();
    }
    int unsat = 0;
    for (int c = threadIdx.x; c < m && !unsat; c += kSynThreads) {
      const int e1 = row_ptr[c + 1];
      uint32_t parity = 0;
      for (int e = row_ptr[c]; e < e1; ++e) {
        const int v = col_idx[e];
        parity ^= STAGE ? zs[v] : (uint32_t)(z[v] != 0);
      }
      unsat = (int)(parity & 1u);
    }
    // Barrier and OR in one: every read of zs for this word is done before the next
    // word's copy overwrites it.
    const int any = __syncthreads_or(unsat);
    if (threadIdx.x == 0) ok[b] = any ? 0 : 1;
  }
}

}  // namespace
}  // namespace ldpc

using namespace ldpc;

extern "C" ldpc_status ldpc_syndrome(ldpc_graph_t g, const uint8_t *hard_bits, int32_t batch, uint8_t *ok,
                                     hipStream_t stream) {
  if (!g) return set_error(LDPC_ERR_INVALID_ARG, "graph is NULL");
  if (batch < 0) return set_error(LDPC_ERR_INVALID_ARG, "batch < 0");
  if (batch == 0) return LDPC_OK;
  if (!hard_bits || !ok) return set_error(LDPC_ERR_INVALID_ARG, "NULL buffer");
  if (g->n <= kSynPackedMaxN) {
    const int32_t groups = batch / kSynWords + (batch % kSynWords != 0);
    const unsigned grid = (unsigned)std::min<int32_t>(groups, kSynMaxGrid);
    const size_t lds = (size_t)g->n * 4;
    const bool vec = (g->n & 3) == 0 && ((uintptr_t)hard_bits & 3) == 0;
    const void *k = vec ? (const void *)syndrome_packed_kernel<true> : (const void *)syndrome_packed_kernel<false>;
    if (lds + 64 > 65536)  // above the default dynamic LDS of a launch (the kernel's own 8 bytes beside it)
      LDPC_HIP_CHECK(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    if (vec)
      hipLaunchKernelGGL(syndrome_packed_kernel<true>, dim3(grid), dim3(kSynThreads), lds, stream, g->d_row_ptr,
                         g->d_col_idx, g->m, g->n, hard_bits, (int)batch, ok);
    else
      hipLaunchKernelGGL(syndrome_packed_kernel<false>, dim3(grid), dim3(kSynThreads), lds, stream, g->d_row_ptr,
                         g->d_col_idx, g->m, g->n, hard_bits, (int)batch, ok);
    LDPC_HIP_CHECK(hipGetLastError());
    return LDPC_OK;
  }
  const unsigned grid = (unsigned)std::min<int32_t>(batch, kSynMaxGrid);
  if (g->n <= kSynLdsMax) {
    const size_t lds = ((size_t)g->n + 15) & ~(size_t)15;
    hipLaunchKernelGGL(syndrome_kernel<true>, dim3(grid), dim3(kSynThreads), lds, stream, g->d_row_ptr, g->d_col_idx,
                       g->m, g->n, hard_bits, (int)batch, ok);
  } else {
    hipLaunchKernelGGL(syndrome_kernel<false>, dim3(grid), dim3(kSynThreads), 0, stream, g->d_row_ptr, g->d_col_idx,
                       g->m, g->n, hard_bits, (int)batch, ok);
  }
  LDPC_HIP_CHECK(hipGetLastError());
  return LDPC_OK;
}
