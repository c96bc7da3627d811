// Plain flooding sum-product decoder: one workgroup per 64-word tile at a time.
//
// The batch is cut into tiles of 64 words (the batch split of Sec. III-C: every
// worker decodes whole words).  A workgroup of W wavefronts owns one tile for the
// whole decode of that tile; its waves split the checks and the variables of the
// graph in the interleaved way of Algorithm 1 (check c and variable v go to wave
// c mod W and v mod W), with a workgroup barrier where Algorithm 1 exchanges messages.
// Workgroups take tiles from a counter and keep one tile state each in the workspace,
// reused from tile to tile, so the workspace holds as many tile states as workgroups
// run at once (at most one per tile), not one per tile of the batch.
//
// HBM state of a tile (all FP32 [index][64]):
//   M  [nnz]  v->c messages (Eq. 6, clamped), stored as M / 16 with the decision z_v
//             (Eq. 8) in the exponent's top bit
//   E0/E1 [nnz] c->v messages of even / odd iterations (Eq. 5)
//   R  [n]  channel LLRs (Eq. 4)
// Iteration t+1 (flooding, Algorithm 1):
//   check phase     every check: syndrome bit of z^(t) (the XOR of its messages' bit 30),
//                   E^(t+1) from M^(t+1) into E[(t+1)&1]
//   decide          a lane whose z^(t) satisfies H z^T = 0 (Eq. 1), or with t = max_iters,
//                   stops at t; from then on nothing of it is written, so its E^(t) stays
//                   in E[t&1]
//   variable phase  every variable: L^(t+1) (Eq. 7), and M^(t+2) (Eq. 6) carrying z^(t+1)
//                   for running lanes
// The egress recomputes each word's final posterior from its own E buffer with the
// same summation as the variable phase, so it equals the L whose decisions stopped it.
//
// State in and out: a decode may start from caller c->v messages E^(0) (placed in E0,
// then one variable phase on them gives L^(0), z^(0) and M^(1)), and may write each
// word's E of its last iteration back out.
#include <mutex>

#include "internal.h"
#include "tile.h"

namespace ldpc {

template <int DC, int DV>
__device__ __forceinline__ void plain_decode_tile(GraphDev g, const float *__restrict__ llr32,
                                                  const double *__restrict__ llr64, int B, int max_iters,
                                                  int early_stop, int tile, const TileState &st,
                                                  uint8_t *__restrict__ hard, float *__restrict__ post,
                                                  int32_t *__restrict__ iters, const float *__restrict__ init_cv,
                                                  float *__restrict__ final_cv, float (*stage)[TW + 1],
                                                  unsigned long long *unsat_w, float *psl) {
  const int lane = lane_id();
  const int wave = wave_id();
  const int W = blockDim.x >> 6;
  const int cw0 = tile * TW;
  const int nvalid = min(TW, B - cw0);

  ingest_tile<DV>(g, llr32, llr64, cw0, nvalid, st, stage, wave, W, lane);
  if (init_cv) {
    ingest_edges(g, init_cv, cw0, nvalid, st.E0, stage, wave, W, lane);
    for (int v = wave; v < g.n; v += W) {
      int p0, dv;
      var_range<DV>(g, v, p0, dv);
      var_update<DV>(st.R, st.E0, st.M, g.var_edges, p0, dv, v, lane, true);
    }
    __syncthreads();
  }

  bool active = lane < nvalid;
  int my_iters = 0;
  for (int it = 0;; ++it) {
    float *En = ((it + 1) & 1) ? st.E1 : st.E0;  // receives E^(it+1)
    int unsat = 0;
    if (active) {  // stopped lanes load nothing
      for (int c = wave; c < g.m; c += W) {
        int e0, dc;
        check_range<DC>(g, c, e0, dc);
        unsat |= check_update<DC>(st.M, En, e0, dc, lane, true, psl);
      }
    }
    const unsigned long long b = __ballot(unsat);
    if (lane == 0) unsat_w[wave] = b;
    __syncthreads();
    unsigned long long um = 0;
    for (int w = 0; w < W; ++w) um |= unsat_w[w];
    const bool lane_unsat = (um >> lane) & 1ull;
    if (active && ((early_stop && !lane_unsat) || it == max_iters)) {
      active = false;
      my_iters = it;
    }
    if (__ballot(active) == 0ull) break;  // same value in every wave of the workgroup
    if (active) {
      for (int v = wave; v < g.n; v += W) {
        int p0, dv;
        var_range<DV>(g, v, p0, dv);
        var_update<DV>(st.R, En, st.M, g.var_edges, p0, dv, v, lane, true);
      }
    }
    __syncthreads();
  }

  egress_tile<DV>(g, st, my_iters, cw0, nvalid, post, hard, stage, wave, W, lane, 0, 1, init_cv != nullptr);
  if (final_cv) egress_edges(g, st, my_iters, init_cv != nullptr, cw0, nvalid, final_cv, stage, wave, W, lane);
  if (wave == 0 && lane < nvalid) iters[cw0 + lane] = my_iters;
}

// Workspace: the tile counter in its first 256 bytes, then one tile state per workgroup.
constexpr size_t kPlainHeader = 256;

template <int DC, int DV>
__device__ __forceinline__ void plain_decode_body(GraphDev g, const float *__restrict__ llr32,
                                                  const double *__restrict__ llr64, int B, int max_iters,
                                                  int early_stop, char *ws, uint8_t *__restrict__ hard,
                                                  float *__restrict__ post, int32_t *__restrict__ iters,
                                                  const float *__restrict__ init_cv, float *__restrict__ final_cv) {
  __shared__ float stage[TW][TW + 1];
  __shared__ unsigned long long unsat_w[16];
  __shared__ int s_tile;
  constexpr int kPsl = check_psl_floats<DC>();  // LDS of high runtime degrees (check_update)
  __shared__ float psl_buf[kPsl > 0 ? 16 * kPsl : 1];
  float *psl = kPsl > 0 ? psl_buf + wave_id() * kPsl : nullptr;
  int *counter = (int *)ws;
  const TileState st =
      tile_state_block(ws + kPlainHeader + (size_t)blockIdx.x * tile_bytes(g.nnz, g.n), g.nnz, g.n);
  const int tiles = (B + TW - 1) / TW;
  for (;;) {
    if (threadIdx.x == 0) s_tile = atomicAdd(counter, 1);
    __syncthreads();
    const int tile = s_tile;
    __syncthreads();  // every thread has read s_tile before thread 0 takes the next one
    if (tile >= tiles) break;  // same value in every thread
    plain_decode_tile<DC, DV>(g, llr32, llr64, B, max_iters, early_stop, tile, st, hard, post, iters, init_cv,
                              final_cv, stage, unsat_w, psl);
    __syncthreads();  // the tile state and the LDS staging are reused by the next tile
  }
}

__global__ void reset_tile_counter(int *counter) {
  if (threadIdx.x == 0) *counter = 0;
}

// Low check degrees fit in 64 VGPRs, so the kernel can ask for 8 waves per SIMD (more
// HBM requests in flight); higher degrees would spill their message arrays to scratch
// under that limit and take the compiler's own register budget instead.
template <int DC, int DV>
constexpr bool plain_fits_8_waves() {
  return DC > 0 ? DC <= 6 : -DC <= 8;
}

template <int DC, int DV>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8)))
    plain_decode_kernel_w8(GraphDev g, const float *__restrict__ llr32, const double *__restrict__ llr64, int B,
                           int max_iters, int early_stop, char *ws, uint8_t *__restrict__ hard,
                           float *__restrict__ post, int32_t *__restrict__ iters, const float *__restrict__ init_cv,
                           float *__restrict__ final_cv) {
  plain_decode_body<DC, DV>(g, llr32, llr64, B, max_iters, early_stop, ws, hard, post, iters, init_cv, final_cv);
}

template <int DC, int DV>
__global__ void __launch_bounds__(1024)
    plain_decode_kernel(GraphDev g, const float *__restrict__ llr32, const double *__restrict__ llr64, int B,
                        int max_iters, int early_stop, char *ws, uint8_t *__restrict__ hard, float *__restrict__ post,
                        int32_t *__restrict__ iters, const float *__restrict__ init_cv, float *__restrict__ final_cv) {
  plain_decode_body<DC, DV>(g, llr32, llr64, B, max_iters, early_stop, ws, hard, post, iters, init_cv, final_cv);
}

}  // namespace ldpc

using namespace ldpc;

namespace {
using PlainKernel = void (*)(GraphDev, const float *, const double *, int, int, int, char *, uint8_t *, float *,
                             int32_t *, const float *, float *);

template <int DC, int DV>
PlainKernel plain_kernel_for() {
  if constexpr (plain_fits_8_waves<DC, DV>())
    return plain_decode_kernel_w8<DC, DV>;
  else
    return plain_decode_kernel<DC, DV>;
}

PlainKernel pick_plain(const ldpc_graph_s *g) {
  PlainKernel k = nullptr;
#define LDPC_PICK(C, V) k = plain_kernel_for<C, V>()
  LDPC_KIND_SWITCH(kernel_kind(g), LDPC_PICK)
#undef LDPC_PICK
  return k;
}

// Workgroups of ldpc_decode's launch shape (16 waves) the current device holds resident at
// once; 0 if the runtime cannot say.
size_t plain_resident_workgroups(const ldpc_graph_s *g) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)pick_plain(g), 1024, 0) != hipSuccess)
    return 0;
  return (size_t)cus * (size_t)per_cu;
}
}  // namespace

size_t plain_workspace_bytes(const ldpc_graph_s *g, int32_t batch) {
  size_t states = ((size_t)batch + TW - 1) / TW;
  const size_t resident = plain_resident_workgroups(g);
  if (resident > 0) states = std::min(states, resident);
  return kPlainHeader + states * tile_bytes(g->nnz, g->n);
}

size_t plain_min_workspace_bytes(const ldpc_graph_s *g) { return kPlainHeader + tile_bytes(g->nnz, g->n); }

ldpc_status launch_plain_decode(const ldpc_graph_s *g, const void *llr, bool llr_f64, int32_t batch,
                                int32_t max_iters, int32_t early_stop, uint8_t *hard, float *post, int32_t *iters,
                                void *ws, size_t ws_bytes, int32_t waves, hipStream_t stream, const float *init_cv,
                                float *final_cv) {
  GraphDev d = graph_dev(g);
  const size_t tiles = ((size_t)batch + TW - 1) / TW;
  const size_t tb = tile_bytes(g->nnz, g->n);
  if (ws_bytes < kPlainHeader + tb) return set_error(LDPC_ERR_INVALID_ARG, "workspace too small");
  // one workgroup per tile state the workspace holds, at most one per tile
  const size_t grid = std::min(tiles, (ws_bytes - kPlainHeader) / tb);
  PlainKernel k = pick_plain(g);
  const float *l32 = llr_f64 ? nullptr : (const float *)llr;
  const double *l64 = llr_f64 ? (const double *)llr : nullptr;
  hipLaunchKernelGGL(reset_tile_counter, dim3(1), dim3(64), 0, stream, (int *)ws);
  LDPC_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(64 * waves), 0, stream, d, l32, l64, (int)batch, (int)max_iters,
                     (int)(early_stop != 0), (char *)ws, hard, post, iters, init_cv, final_cv);
  LDPC_HIP_CHECK(hipGetLastError());
  return LDPC_OK;
}

// ---- allocation-free entry point ----------------------------------------------------
//
// The tile state of ldpc_decode_noalloc lives in a fixed array in device memory that the
// library's code object holds on every GPU it is loaded on (LDPC_NOALLOC_SCRATCH_BYTES).
// Host code must not use the array's name as an address: each device's copy is found
// once with hipGetSymbolAddress (with that device current) and that pointer is what the
// kernels receive.
static __device__ __align__(256) unsigned char scratch[LDPC_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

ldpc_status scratch_for_current_device(void **out) {
  int dev = 0;
  LDPC_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return set_error(LDPC_ERR_DEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
    if (!p) return set_error(LDPC_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LDPC_OK;
}
}  // namespace

extern "C" ldpc_status ldpc_decode_noalloc(ldpc_graph_t g, const void *llr, int32_t batch, int32_t max_iters,
                                           int32_t early_stop, uint32_t flags, uint8_t *hard_bits, float *posterior,
                                           int32_t *iters_used, hipStream_t stream) {
  if (!g) return set_error(LDPC_ERR_INVALID_ARG, "graph is NULL");
  if (batch < 0) return set_error(LDPC_ERR_INVALID_ARG, "batch < 0");
  if (max_iters < 0) return set_error(LDPC_ERR_INVALID_ARG, "max_iters < 0");
  if (flags & ~LDPC_LLR_F64) return set_error(LDPC_ERR_INVALID_ARG, "unknown flag");
  if (batch == 0) return LDPC_OK;
  if (!llr || !hard_bits || !posterior || !iters_used) return set_error(LDPC_ERR_INVALID_ARG, "NULL buffer");
  const size_t need = plain_workspace_bytes(g, batch);
  if (need > (size_t)LDPC_NOALLOC_SCRATCH_BYTES)
    return set_error(LDPC_ERR_INVALID_ARG,
                     "batch needs " + std::to_string(need) + " bytes of tile state, above the fixed " +
                         std::to_string((size_t)LDPC_NOALLOC_SCRATCH_BYTES) + "-byte scratch (at most " +
                         std::to_string(LDPC_NOALLOC_SCRATCH_BYTES / tile_bytes(g->nnz, g->n) * kTile) +
                         " words of this code per call)");
  void *ws = nullptr;
  ldpc_status st = scratch_for_current_device(&ws);
  if (st != LDPC_OK) return st;
  // 16 waves per tile, as ldpc_decode
  return launch_plain_decode(g, llr, (flags & LDPC_LLR_F64) != 0, batch, max_iters, early_stop, hard_bits, posterior,
                             iters_used, ws, (size_t)LDPC_NOALLOC_SCRATCH_BYTES, 16, stream);
}
