// Syndrome test of Eq. 1 on given hard decisions: ok[b] = 1 iff every check of H
// sees an even number of ones among word b's decisions (H z_b^T = 0 over GF(2)).
//
// The decoders apply this test inside their iterations to stop a word early; this
// entry point applies it to any batch of decisions (a decoder's output after a run
// without early stop, or words from elsewhere), so that a caller can tell a word that
// satisfies every check at the iteration limit from one that does not.
//
// One workgroup per word, taken in grid-stride order.  Words of up to kSynLdsMax bits
// are first copied to LDS (one coalesced pass over the row), then each thread takes
// checks c = tid, tid + 256, ... and gathers the decisions of the check's variables
// from there; longer words are gathered from global memory, where L1/L2 hold the row.
// A thread stops at its first unsatisfied check; the workgroup ORs its threads' results
// with one barrier.  The cost is one read of the decisions (n bytes per word).
#include <algorithm>

#include "internal.h"

namespace ldpc {
namespace {

constexpr int kSynThreads = 256;
constexpr int kSynLdsMax = 65536;      // bytes of LDS a workgroup may use without opt-in
constexpr int kSynMaxGrid = 256 * 32;  // workgroups per launch (words beyond are strided)

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
