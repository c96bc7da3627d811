// Stream form: one word per workgroup, the whole decoding state in LDS.
//
// Sec. III-B spreads one word's Tanner graph over many workers ("stream
// processing") and finds the exchange of messages between workers, every
// half-iteration, to be its cost.  Inside one compute unit that exchange is an
// LDS barrier, so here a workgroup owns one word at a time: its threads take
// the checks (check phase) and then the variables (variable phase), in the
// interleaved order of Algorithm 1 (check c and variable v on thread c mod NT and
// v mod NT), and every message stays in LDS.  Workgroups are persistent and take
// the next word from an atomic counter when theirs stops, so a word that needs
// few iterations never waits for another.
//
// LDS per word (all indexed in check-major edge order):
//   M  [nnz] FP32 v->c messages (Eq. 6, clamped)    E [nnz] FP32 c->v messages (Eq. 5)
//   Z  [nnz] u8   decision of each edge's variable   R, L [n] FP32 channel LLRs, posterior
// The check phase tests the syndrome of the decisions it reads (Eq. 1) while it
// computes new messages; the posterior of the last variable phase stays in L.
// Per edge the arithmetic and its order are those of the plain decoder, so the
// outputs are identical to it bit for bit.
#include "internal.h"
#include "tile.h"

namespace ldpc {

__host__ __device__ inline size_t stream_lds_bytes(int64_t nnz, int32_t n) {
  return (size_t)nnz * 9 + (size_t)n * 8 + 16;
}

// Workgroup size limit per degree pair: the generic kernels for check degrees above 8
// hold up to 32 messages per thread and would spill under the 128-VGPR budget of a
// 1024-thread workgroup, so they are built for at most 512 threads (256 VGPRs).
template <int DC>
constexpr int kStreamMaxThreads = DC < -8 ? 512 : 1024;

template <int DC, int DV>
__global__ void __launch_bounds__(kStreamMaxThreads<DC>)
    stream_decode_kernel(GraphDev g, const float *__restrict__ llr32, const double *__restrict__ llr64, int B,
                         int max_iters, int early_stop, int *counter, uint8_t *__restrict__ hard,
                         float *__restrict__ post, int32_t *__restrict__ iters) {
  constexpr int DCM = DC > 0 ? DC : -DC;
  constexpr int DVM = DV > 0 ? DV : -DV;
  extern __shared__ float smem[];
  __shared__ int s_word;
  float *Mv = smem;
  float *Ec = Mv + g.nnz;
  float *R = Ec + g.nnz;
  float *L = R + g.n;
  uint8_t *Zb = (uint8_t *)(L + g.n);
  const int t = threadIdx.x, NT = blockDim.x;
  const size_t n = (size_t)g.n;

  for (;;) {
    if (t == 0) s_word = atomicAdd(counter, 1);
    __syncthreads();
    const int word = s_word;
    if (word >= B) break;  // same value in every thread

    // ingest: R = L = channel LLRs, first messages M = clamp(R), channel decisions
    for (int v = t; v < g.n; v += NT) {
      const size_t off = (size_t)word * n + (size_t)v;
      const float x = llr64 ? (float)llr64[off] : llr32[off];
      R[v] = x;
      L[v] = x;
      int p0, dv;
      var_range<DV>(g, v, p0, dv);
      const float mx = clamp_msg(x);
      const uint8_t z = x <= 0.0f ? 1 : 0;
      for (int j = 0; j < dv; ++j) {
        const int e = g.var_edges[p0 + j];
        Mv[e] = mx;
        Zb[e] = z;
      }
    }
    __syncthreads();

    int it = 0;
    for (;;) {
      int unsat = 0;
      for (int c = t; c < g.m; c += NT) {
        int e0, dc;
        check_range<DC>(g, c, e0, dc);
        float mv[DCM], ev[DCM];
        int par = 0;
#pragma unroll
        for (int j = 0; j < DCM; ++j) {
          if (DC > 0 || j < dc) {
            mv[j] = Mv[e0 + j];
            par ^= Zb[e0 + j];
          }
        }
        check_core<DC>(mv, dc, ev);
#pragma unroll
        for (int j = 0; j < DCM; ++j)
          if (DC > 0 || j < dc) Ec[e0 + j] = ev[j];
        unsat |= par;
      }
      const int any_unsat = __syncthreads_or(unsat);
      if ((early_stop && !any_unsat) || it == max_iters) break;  // same value in every thread
      for (int v = t; v < g.n; v += NT) {
        int p0, dv;
        var_range<DV>(g, v, p0, dv);
        float ev[DVM], pre[DVM];
        int eid[DVM];
        const float r = R[v];
#pragma unroll
        for (int j = 0; j < DVM; ++j) {
          if (DV > 0 || j < dv) {
            eid[j] = g.var_edges[p0 + j];
            ev[j] = Ec[eid[j]];
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
        L[v] = acc;
        const uint8_t z = acc <= 0.0f ? 1 : 0;
        float suf = 0.0f;
#pragma unroll
        for (int j = DVM - 1; j >= 0; --j) {
          if (DV > 0 || j < dv) {
            Mv[eid[j]] = clamp_msg(pre[j] + suf);
            Zb[eid[j]] = z;
            suf += ev[j];
          }
        }
      }
      __syncthreads();
      ++it;
    }

    for (int v = t; v < g.n; v += NT) {
      const float x = L[v];
      const size_t off = (size_t)word * n + (size_t)v;
      post[off] = x;
      hard[off] = x <= 0.0f ? 1 : 0;
    }
    if (t == 0) iters[word] = it;
    __syncthreads();  // L and s_word are reused by the next word
  }
}

__global__ void reset_counter(int *counter) {
  if (threadIdx.x == 0) *counter = 0;
}

}  // namespace ldpc

using namespace ldpc;

namespace {
using StreamKernel = void (*)(GraphDev, const float *, const double *, int, int, int, int *, uint8_t *, float *,
                              int32_t *);

StreamKernel pick_stream(const ldpc_graph_s *g, int &max_threads) {
  StreamKernel k = nullptr;
#define LDPC_PICK(C, V)                    \
  k = stream_decode_kernel<C, V>;          \
  max_threads = kStreamMaxThreads<C>
  LDPC_KIND_SWITCH(kernel_kind(g), LDPC_PICK)
#undef LDPC_PICK
  return k;
}

int stream_threads(const ldpc_graph_s *g, int max_threads) {
  const int big = std::max(g->m, g->n);
  int nt = 64;
  while (nt < max_threads && nt * 2 <= big) nt *= 2;
  return nt;
}
}  // namespace

extern "C" ldpc_status ldpc_stream_lds_bytes(ldpc_graph_t g, size_t *bytes, int32_t *supported) {
  if (!g) return set_error(LDPC_ERR_INVALID_ARG, "graph is NULL");
  const size_t b = stream_lds_bytes(g->nnz, g->n);
  if (bytes) *bytes = b;
  if (supported) {
    int dev = 0, lim = 0;
    LDPC_HIP_CHECK(hipGetDevice(&dev));
    LDPC_HIP_CHECK(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    *supported = b + 64 <= (size_t)lim ? 1 : 0;
  }
  return LDPC_OK;
}

extern "C" ldpc_status ldpc_decode_stream(ldpc_graph_t g, const void *llr, int32_t batch, int32_t max_iters,
                                          int32_t early_stop, uint32_t flags, uint8_t *hard_bits, float *posterior,
                                          int32_t *iters_used, void *workspace, size_t ws_bytes, int32_t threads,
                                          hipStream_t stream) {
  if (!g) return set_error(LDPC_ERR_INVALID_ARG, "graph is NULL");
  if (batch < 0 || max_iters < 0) return set_error(LDPC_ERR_INVALID_ARG, "negative batch or max_iters");
  if (flags & ~LDPC_LLR_F64) return set_error(LDPC_ERR_INVALID_ARG, "unknown flag");
  if (threads != 0 && (threads < 64 || threads > 1024 || threads % 64))
    return set_error(LDPC_ERR_INVALID_ARG, "threads must be 0 or a multiple of 64 in 64..1024");
  if (batch == 0) return LDPC_OK;
  if (!llr || !hard_bits || !posterior || !iters_used || !workspace)
    return set_error(LDPC_ERR_INVALID_ARG, "NULL buffer");
  if (ws_bytes < 256) return set_error(LDPC_ERR_INVALID_ARG, "workspace too small (256 bytes)");
  size_t lds = 0;
  int32_t ok = 0;
  ldpc_status st = ldpc_stream_lds_bytes(g, &lds, &ok);
  if (st != LDPC_OK) return st;
  if (!ok) return set_error(LDPC_ERR_UNSUPPORTED, "word state (" + std::to_string(lds) + " bytes) exceeds LDS");
  int max_threads = 1024;
  StreamKernel k = pick_stream(g, max_threads);
  if (threads > max_threads)
    return set_error(LDPC_ERR_INVALID_ARG,
                     "threads above " + std::to_string(max_threads) + " for this code's check degree");
  const int nt = threads ? threads : stream_threads(g, max_threads);
  int dev = 0, cus = 0, per_cu = 0;
  LDPC_HIP_CHECK(hipGetDevice(&dev));
  LDPC_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  LDPC_HIP_CHECK(hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  LDPC_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k, nt, lds));
  if (per_cu < 1) return set_error(LDPC_ERR_UNSUPPORTED, "stream kernel cannot be resident");
  const int grid = std::min(batch, cus * per_cu);
  int *counter = (int *)workspace;
  hipLaunchKernelGGL(reset_counter, dim3(1), dim3(64), 0, stream, counter);
  LDPC_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k, dim3(grid), dim3(nt), lds, stream, graph_dev(g), (flags & LDPC_LLR_F64) ? nullptr : (const float *)llr,
                     (flags & LDPC_LLR_F64) ? (const double *)llr : nullptr, (int)batch, (int)max_iters,
                     (int)(early_stop != 0), counter, hard_bits, posterior, iters_used);
  LDPC_HIP_CHECK(hipGetLastError());
  return LDPC_OK;
}
