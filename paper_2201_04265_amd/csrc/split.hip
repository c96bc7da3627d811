// Split form of the plain decoder, for batches with few 64-word tiles.
//
// The plain decoder gives each tile one workgroup for the whole decode, so a batch
// of a few hundred words of a long code keeps a handful of compute units busy.
// Here every half-iteration of Algorithm 1 is its own launch, and each launch
// spreads one tile's checks (or variables) over many workgroups ("slices"); the
// launch boundary is the exchange of messages that Algorithm 1 places between the
// check and the variable phases.  Tile state, arithmetic and the per-lane stopping
// rule are those of the plain decoder (same device functions, same order), so the
// outputs are identical to ldpc_decode bit for bit.
//
// Per tile a control block holds the running lanes and the syndrome bits, each
// double-buffered by iteration parity so that the slices of one launch read one
// buffer while slice 0 prepares the other:
//   active[it & 1]  lanes still decoding when iteration it's check phase runs
//   unsat[it & 1]   lanes whose decisions z^(it) leave a check unsatisfied (Eq. 1),
//                   ORed in by the check phase of iteration it
//   iters[64]       iterations used by each lane
// Launches for it = 0 .. max_iters: check(it) then decide-and-variable(it); a tile
// whose lanes have all stopped returns at once, so the remaining launches cost
// only their dispatch.
#include "internal.h"
#include "tile.h"

namespace ldpc {

struct SplitCtl {
  unsigned long long active[2];
  unsigned long long unsat[2];
  int32_t iters[TW];
};
constexpr size_t kSplitCtlBytes = 512;
static_assert(sizeof(SplitCtl) <= kSplitCtlBytes, "control block");
constexpr int kSplitWaves = 8;

__host__ __device__ inline size_t split_tiles(int32_t batch) { return ((size_t)batch + TW - 1) / TW; }

// Ingest and egress move 64-variable chunks of a tile through LDS; the slices of a
// tile take every slices-th chunk.
template <int DV>
__global__ void __launch_bounds__(64 * kSplitWaves)
    split_ingest_kernel(GraphDev g, const float *__restrict__ llr32, const double *__restrict__ llr64, int B,
                        char *ws, SplitCtl *ctl, int slices) {
  __shared__ float stage[TW][TW + 1];
  const int lane = lane_id(), wave = wave_id(), W = blockDim.x >> 6;
  const int tile = blockIdx.x / slices, s = blockIdx.x - tile * slices;
  const int cw0 = tile * TW;
  const int nvalid = min(TW, B - cw0);
  const TileState st = tile_state_block(ws + (size_t)tile * tile_bytes(g.nnz, g.n), g.nnz, g.n);
  ingest_tile<DV>(g, llr32, llr64, cw0, nvalid, st, stage, wave, W, lane, s, slices);
  SplitCtl &c = ctl[tile];
  if (s == 0 && wave == 0) {
    c.iters[lane] = 0;
    if (lane == 0) {
      c.active[0] = nvalid == TW ? ~0ull : ((1ull << nvalid) - 1ull);
      c.active[1] = 0ull;
      c.unsat[0] = 0ull;
      c.unsat[1] = 0ull;
    }
  }
}

// Check phase of iteration it: E^(it+1) from M, syndrome bits of z^(it).
template <int DC>
__global__ void __launch_bounds__(64 * kSplitWaves)
    split_check_kernel(GraphDev g, char *ws, SplitCtl *ctl, int it, int slices) {
  const int lane = lane_id(), wave = wave_id(), W = blockDim.x >> 6;
  constexpr int kPsl = check_psl_floats<DC>();  // LDS of high runtime degrees (check_update)
  __shared__ float psl_buf[kPsl > 0 ? kSplitWaves * kPsl : 1];
  const int tile = blockIdx.x / slices, s = blockIdx.x - tile * slices;
  SplitCtl &c = ctl[tile];
  const unsigned long long act = c.active[it & 1];
  if (act == 0ull) return;  // same value in the whole workgroup
  const bool active = (act >> lane) & 1ull;
  const TileState st = tile_state_block(ws + (size_t)tile * tile_bytes(g.nnz, g.n), g.nnz, g.n);
  float *En = ((it + 1) & 1) ? st.E1 : st.E0;
  int unsat = 0;
  for (int ch = s * W + wave; ch < g.m; ch += slices * W) {
    int e0, dc;
    check_range<DC>(g, ch, e0, dc);
    unsat |= check_update<DC>(st.M, En, e0, dc, lane, active, kPsl > 0 ? psl_buf + wave * kPsl : nullptr);
  }
  const unsigned long long b = __ballot(unsat);
  if (lane == 0 && b) atomicOr(&c.unsat[it & 1], b);
}

// Decision of iteration it (a lane stops at the first zero syndrome, or at max_iters),
// then the variable phase for the lanes still running: L^(it+1) and M^(it+2).
template <int DV>
__global__ void __launch_bounds__(64 * kSplitWaves)
    split_var_kernel(GraphDev g, char *ws, SplitCtl *ctl, int it, int max_iters, int early_stop, int slices) {
  const int lane = lane_id(), wave = wave_id(), W = blockDim.x >> 6;
  const int tile = blockIdx.x / slices, s = blockIdx.x - tile * slices;
  SplitCtl &c = ctl[tile];
  const unsigned long long act = c.active[it & 1];
  const unsigned long long um = c.unsat[it & 1];
  const bool was = (act >> lane) & 1ull;
  const bool stop = was && ((early_stop && !((um >> lane) & 1ull)) || it == max_iters);
  const bool still = was && !stop;
  const unsigned long long nact = __ballot(still);
  if (s == 0 && wave == 0) {  // the only writer of the control block in this launch
    if (stop) c.iters[lane] = it;
    if (lane == 0) {
      c.active[(it + 1) & 1] = nact;
      c.unsat[(it + 1) & 1] = 0ull;
    }
  }
  if (nact == 0ull) return;
  const TileState st = tile_state_block(ws + (size_t)tile * tile_bytes(g.nnz, g.n), g.nnz, g.n);
  const float *En = ((it + 1) & 1) ? st.E1 : st.E0;
  for (int v = s * W + wave; v < g.n; v += slices * W) {
    int p0, dv;
    var_range<DV>(g, v, p0, dv);
    var_update<DV>(st.R, En, st.M, g.var_edges, p0, dv, v, lane, still);
  }
}

template <int DV>
__global__ void __launch_bounds__(64 * kSplitWaves)
    split_egress_kernel(GraphDev g, char *ws, const SplitCtl *ctl, int B, float *__restrict__ post,
                        uint8_t *__restrict__ hard, int32_t *__restrict__ iters, int slices) {
  __shared__ float stage[TW][TW + 1];
  const int lane = lane_id(), wave = wave_id(), W = blockDim.x >> 6;
  const int tile = blockIdx.x / slices, s = blockIdx.x - tile * slices;
  const int cw0 = tile * TW;
  const int nvalid = min(TW, B - cw0);
  const TileState st = tile_state_block(ws + (size_t)tile * tile_bytes(g.nnz, g.n), g.nnz, g.n);
  const int my_iters = ctl[tile].iters[lane];
  egress_tile<DV>(g, st, my_iters, cw0, nvalid, post, hard, stage, wave, W, lane, s, slices);
  if (s == 0 && wave == 0 && lane < nvalid) iters[cw0 + lane] = my_iters;
}

}  // namespace ldpc

using namespace ldpc;

size_t split_workspace_bytes(const ldpc_graph_s *g, int32_t batch) {
  const size_t tiles = split_tiles(batch);
  return tiles * tile_bytes(g->nnz, g->n) + align256(tiles * kSplitCtlBytes);
}

namespace {

struct SplitKernels {
  void (*ingest)(GraphDev, const float *, const double *, int, char *, SplitCtl *, int);
  void (*check)(GraphDev, char *, SplitCtl *, int, int);
  void (*var)(GraphDev, char *, SplitCtl *, int, int, int, int);
  void (*egress)(GraphDev, char *, const SplitCtl *, int, float *, uint8_t *, int32_t *, int);
};

SplitKernels pick_split(const ldpc_graph_s *g) {
  SplitKernels k{};
#define LDPC_PICK(C, V)                \
  k.ingest = split_ingest_kernel<V>;   \
  k.check = split_check_kernel<C>;     \
  k.var = split_var_kernel<V>;         \
  k.egress = split_egress_kernel<V>
  LDPC_KIND_SWITCH(kernel_kind(g), LDPC_PICK)
#undef LDPC_PICK
  return k;
}

// Workgroups per tile in the phase launches: about 2048 workgroups in all, and at
// least 4 checks or variables per wave.
int split_slices(const ldpc_graph_s *g, size_t tiles) {
  const long per_tile_max = std::max<long>(1, (std::max(g->m, g->n) + 4 * kSplitWaves - 1) / (4 * kSplitWaves));
  const long want = (2048 + (long)tiles - 1) / (long)tiles;
  return (int)std::max<long>(1, std::min(want, per_tile_max));
}

}  // namespace

ldpc_status launch_split_decode(const ldpc_graph_s *g, const void *llr, bool llr_f64, int32_t batch,
                                int32_t max_iters, int32_t early_stop, uint8_t *hard, float *post, int32_t *iters,
                                void *ws, int32_t slices, hipStream_t stream) {
  if (batch == 0) return LDPC_OK;
  const size_t tiles = split_tiles(batch);
  if (slices <= 0) slices = split_slices(g, tiles);
  if ((size_t)slices * tiles > (size_t)INT32_MAX) return set_error(LDPC_ERR_INVALID_ARG, "too many slices");
  const SplitKernels k = pick_split(g);
  const GraphDev d = graph_dev(g);
  char *states = (char *)ws;
  SplitCtl *ctl = (SplitCtl *)(states + tiles * tile_bytes(g->nnz, g->n));
  const float *l32 = llr_f64 ? nullptr : (const float *)llr;
  const double *l64 = llr_f64 ? (const double *)llr : nullptr;
  const dim3 block(64 * kSplitWaves);
  const int cslices = std::min(slices, (g->n + TW - 1) / TW);  // ingest / egress: at most one chunk each
  hipLaunchKernelGGL(k.ingest, dim3((unsigned)(tiles * cslices)), block, 0, stream, d, l32, l64, (int)batch, states,
                     ctl, cslices);
  LDPC_HIP_CHECK(hipGetLastError());
  const dim3 grid((unsigned)(tiles * slices));
  for (int it = 0; it <= max_iters; ++it) {
    hipLaunchKernelGGL(k.check, grid, block, 0, stream, d, states, ctl, it, slices);
    hipLaunchKernelGGL(k.var, grid, block, 0, stream, d, states, ctl, it, (int)max_iters, (int)(early_stop != 0),
                       slices);
  }
  LDPC_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k.egress, dim3((unsigned)(tiles * cslices)), block, 0, stream, d, states,
                     (const SplitCtl *)ctl, (int)batch, post, hard, iters, cslices);
  LDPC_HIP_CHECK(hipGetLastError());
  return LDPC_OK;
}

extern "C" ldpc_status ldpc_split_workspace_size(ldpc_graph_t g, int32_t batch, size_t *bytes) {
  if (!g || !bytes) return set_error(LDPC_ERR_INVALID_ARG, "graph or bytes is NULL");
  if (batch < 0) return set_error(LDPC_ERR_INVALID_ARG, "batch < 0");
  *bytes = split_workspace_bytes(g, batch);
  return LDPC_OK;
}

extern "C" ldpc_status ldpc_decode_split(ldpc_graph_t g, const void *llr, int32_t batch, int32_t max_iters,
                                         int32_t early_stop, uint32_t flags, uint8_t *hard_bits, float *posterior,
                                         int32_t *iters_used, void *workspace, size_t ws_bytes, int32_t slices,
                                         hipStream_t stream) {
  if (!g) return set_error(LDPC_ERR_INVALID_ARG, "graph is NULL");
  if (batch < 0 || max_iters < 0) return set_error(LDPC_ERR_INVALID_ARG, "negative batch or max_iters");
  if (flags & ~LDPC_LLR_F64) return set_error(LDPC_ERR_INVALID_ARG, "unknown flag");
  if (slices < 0) return set_error(LDPC_ERR_INVALID_ARG, "slices < 0");
  if (batch == 0) return LDPC_OK;
  if (!llr || !hard_bits || !posterior || !iters_used || !workspace)
    return set_error(LDPC_ERR_INVALID_ARG, "NULL buffer");
  if (((uintptr_t)workspace & 255) != 0) return set_error(LDPC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < split_workspace_bytes(g, batch)) return set_error(LDPC_ERR_INVALID_ARG, "workspace too small");
  return launch_split_decode(g, llr, (flags & LDPC_LLR_F64) != 0, batch, max_iters, early_stop, hard_bits, posterior,
                             iters_used, workspace, slices, stream);
}
