// Batched persistent decoder: several codes, one launch, per-word refill.
//
// Sec. III-C distributes a batch of whole words over workers that decode them
// one after another.  Here a worker is a "slot": one workgroup holding the
// state of 64 words (one per lane) of a single code, with the same tile layout
// and the same check / variable updates as the plain decoder.  A lane whose word
// stops (zero syndrome or max_iters) writes that word's outputs and claims the
// next word of its code from a per-code atomic counter (one atomic per
// wavefront per refill), so no lane waits for the slowest word of a tile.  All
// codes of a batch run in one launch: workgroup i serves the code whose slot
// range contains i.  Per word the arithmetic and its order are those of the
// plain decoder, so outputs are bit-identical to it whatever lane or slot ran
// the word.
//
// Step G of a slot: check phase writes E into E[(G+1)&1] and tests the
// syndrome of the decisions the messages carry; lanes that stop at G have their last messages in
// E[G&1] (all lanes of a slot share the step parity, so buffer choice is uniform).
#include <cmath>

#include "internal.h"
#include "multi.h"
#include "tile.h"

namespace ldpc {

// Channel LLRs of fresh words into R (the variable phase then derives their first
// messages and decisions with all incoming messages taken as 0).  A stopped word's
// outputs are recomputed from its last messages, which nothing overwrites while it
// waits: its lane's check-phase stores are masked off from the step it stops.
__device__ __forceinline__ void ingest_lanes(const GraphDev &g, const float *__restrict__ llr, TileState st, int word,
                                             bool fresh, int wave, int W, int lane) {
  if (!fresh) return;
  const float *src = llr + (size_t)word * (size_t)g.n;
  for (int v = wave; v < g.n; v += W) st.R[v * TW + lane] = src[v];
}

// Outputs of the lanes in `out`: the posterior of their last iteration, recomputed
// from their last messages (in E1 when `odd`, else E0; R itself when they stopped
// before any iteration) with the variable phase's summation order, and its
// decisions, straight into the word's row of [B][n].
template <int DV>
__device__ __forceinline__ void egress_lanes(const GraphDev &g, TileState st, int word, bool out, bool odd,
                                             int it_lane, float *__restrict__ post, uint8_t *__restrict__ hard,
                                             int wave, int W, int lane) {
  constexpr int DMAX = DV > 0 ? DV : -DV;
  if (!out) return;
  const float *Ep = odd ? st.E1 : st.E0;
  float *prow = post + (size_t)word * (size_t)g.n;
  uint8_t *hrow = hard + (size_t)word * (size_t)g.n;
  for (int v = wave; v < g.n; v += W) {
    int p0, dv;
    var_range<DV>(g, v, p0, dv);
    float L = st.R[v * TW + lane];
    if (it_lane > 0) {  // the variable phase's own sum (var_posterior)
      float ev[DMAX];
      int eid[DMAX];
      L = (float)var_posterior<DV>(L, Ep, g.var_edges, p0, dv, lane, ev, eid);
    }
    prow[v] = L;
    hrow[v] = L <= 0.0f ? 1 : 0;
  }
}

__device__ __forceinline__ int next_word(const MultiJob &J, int w) {
  return w < J.batch ? (J.order ? J.order[w] : w) : -1;
}

// Variable phase of a slot: running lanes update, fresh lanes initialise.
template <int DV>
__device__ __forceinline__ void slot_var_phase(const GraphDev &g, TileState st, const float *En, bool running,
                                               bool fresh, int wave, int W, int lane) {
  if (!(running || fresh)) return;  // idle lanes load nothing
  for (int v = wave; v < g.n; v += W) {
    int p0, dv;
    var_range<DV>(g, v, p0, dv);
    var_update<DV, true>(st.R, En, st.M, g.var_edges, p0, dv, v, lane, true, fresh);
  }
}

// One slot: lanes take words of job J until its queue is empty.  A lane whose
// word stops becomes pending; pending lanes are written out and refilled together
// once at least `refill_min` of them wait or no lane is running.
template <int DC, int DV>
__device__ void run_slot(const MultiJob &J, int local_slot, int *counter, int early_stop, int refill_min, int lanes,
                         unsigned long long *unsat_w, int *lane_word, int wave, int W, int lane, float *psl) {
  const GraphDev &g = J.g;
  const TileState st = tile_state_block(J.ws + (size_t)local_slot * tile_bytes(g.nnz, g.n), g.nnz, g.n);

  if (wave == 0) {  // lanes >= `lanes` never take a word
    int base = 0;
    if (lane == 0) base = atomicAdd(counter, lanes);
    base = __shfl(base, 0);
    lane_word[lane] = lane < lanes ? next_word(J, base + lane) : -1;
  }
  __syncthreads();
  int word = lane_word[lane];
  bool has = word >= 0;  // lane holds a word (running or pending)
  bool pending = false;  // its word has stopped and waits for output
  bool odd = false;      // its last messages are in E1 (else E0)
  int it_lane = 0;
  if (__ballot(has) == 0ull) return;  // uniform: nothing left for this slot
  ingest_lanes(g, J.llr, st, word, has, wave, W, lane);
  slot_var_phase<DV>(g, st, st.E0, false, has, wave, W, lane);
  __syncthreads();

  for (int G = 0;; ++G) {
    float *En = ((G + 1) & 1) ? st.E1 : st.E0;
    const bool active = has && !pending;
    int unsat = 0;
    if (active) {  // idle and stopped lanes load nothing
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
    const bool stop = active && ((early_stop && !lane_unsat) || it_lane == J.max_iters);
    if (stop) odd = (G & 1) != 0;  // E^(it) was written at step G-1 into E[G & 1]
    pending = pending || stop;
    const bool running = active && !stop;
    const unsigned long long pmask = __ballot(pending);
    const unsigned long long rmask = __ballot(running);
    bool fresh = false;
    if (pmask != 0ull && (__popcll(pmask) >= refill_min || rmask == 0ull)) {  // same in every wave
      egress_lanes<DV>(g, st, word, pending, odd, it_lane, J.post, J.hard, wave, W, lane);
      if (wave == 0) {
        if (pending) J.iters[word] = it_lane;
        int base = 0;
        if (lane == 0) base = atomicAdd(counter, __popcll(pmask));
        base = __shfl(base, 0);
        const int rank = __popcll(pmask & ((1ull << lane) - 1ull));
        lane_word[lane] = pending ? next_word(J, base + rank) : word;
      }
      __syncthreads();
      const int nw = lane_word[lane];
      fresh = pending && nw >= 0;
      if (pending) {
        word = nw;
        has = nw >= 0;
        it_lane = 0;
        pending = false;
      }
      ingest_lanes(g, J.llr, st, word, fresh, wave, W, lane);
    }
    if (__ballot(has) == 0ull) break;  // same value in every wave
    slot_var_phase<DV>(g, st, En, running, fresh, wave, W, lane);
    if (running) ++it_lane;
    __syncthreads();
  }
}

__device__ __forceinline__ int find_job(const MultiArgs &a, int slot) {
  int q = 0;
  for (int i = 0; i < a.njobs; ++i)
    if (slot >= a.jobs[i].slot0) q = i;
  return q;
}

template <int DC, int DV>
__global__ void __launch_bounds__(1024) multi_kernel_single(MultiArgs a, int *counters, int early_stop) {
  __shared__ unsigned long long unsat_w[16];
  __shared__ int lane_word[TW];
  constexpr int kPsl = check_psl_floats<DC>();  // LDS of high runtime degrees (check_update)
  __shared__ float psl_buf[kPsl > 0 ? 16 * kPsl : 1];
  const int slot = blockIdx.x;
  const int q = find_job(a, slot);
  run_slot<DC, DV>(a.jobs[q], slot - a.jobs[q].slot0, counters + q, early_stop, a.refill_min, a.lanes, unsat_w,
                   lane_word,
                   wave_id(), blockDim.x >> 6, lane_id(), kPsl > 0 ? psl_buf + wave_id() * kPsl : nullptr);
}

// Codes of different degree profiles in one launch: the generic (runtime degree)
// path for every code, with the largest check degree of the batch as the bound.
template <int DC>
__global__ void __launch_bounds__(1024) multi_kernel_mixed(MultiArgs a, int *counters, int early_stop) {
  __shared__ unsigned long long unsat_w[16];
  __shared__ int lane_word[TW];
  constexpr int kPsl = check_psl_floats<DC>();  // LDS of high runtime degrees (check_update)
  __shared__ float psl_buf[kPsl > 0 ? 16 * kPsl : 1];
  const int slot = blockIdx.x;
  const int q = find_job(a, slot);
  run_slot<DC, -LDPC_MAX_VAR_DEGREE>(a.jobs[q], slot - a.jobs[q].slot0, counters + q, early_stop, a.refill_min,
                                     a.lanes, unsat_w, lane_word, wave_id(), blockDim.x >> 6, lane_id(),
                                     kPsl > 0 ? psl_buf + wave_id() * kPsl : nullptr);
}

__global__ void reset_counters(int *counters, int n) {
  if ((int)threadIdx.x < n) counters[threadIdx.x] = 0;
}

}  // namespace ldpc

using namespace ldpc;

namespace {

using MultiKernel = void (*)(MultiArgs, int *, int);

MultiKernel pick_single(int32_t kind) {
  MultiKernel k = nullptr;
#define LDPC_PICK(C, V) k = multi_kernel_single<C, V>
  LDPC_KIND_SWITCH(kind, LDPC_PICK)
#undef LDPC_PICK
  return k;
}

}  // namespace

// The kernel for the codes that have slots (codes decoded elsewhere, e.g. in the stream
// form, do not force the generic mixed kernel on the others).
MultiKernel multi_kernel_for(const MultiArgs &a) {
  bool any = false;
  for (int i = 0; i < a.njobs; ++i) any |= a.jobs[i].nslots > 0;
  bool same = true;
  int dcmax = 0, kind = -1;
  for (int i = 0; i < a.njobs; ++i) {
    if (any && a.jobs[i].nslots == 0) continue;
    if (kind < 0) kind = a.jobs[i].kind;
    same &= a.jobs[i].kind == kind;
    dcmax = std::max(dcmax, a.jobs[i].dc_max);
  }
  if (same) return pick_single(kind);
  if (dcmax <= 16) return multi_kernel_mixed<-16>;
  if (dcmax <= 24) return multi_kernel_mixed<-24>;
  return multi_kernel_mixed<-LDPC_MAX_CHECK_DEGREE>;
}

ldpc_status multi_resolve(const ldpc_graph_t *graphs, int32_t ncodes, const ldpc_job *jobs,
                          const ldpc_multi_shape *shape_in, ldpc_multi_shape *shape_out, size_t *ws_bytes) {
  if (!graphs || !jobs || ncodes < 1 || ncodes > LDPC_MAX_CODES)
    return set_error(LDPC_ERR_INVALID_ARG, "need 1.." + std::to_string(LDPC_MAX_CODES) + " codes");
  ldpc_multi_shape sh{};
  if (shape_in) sh = *shape_in;
  for (int q = 0; q < ncodes; ++q)
    if (!graphs[q]) return set_error(LDPC_ERR_INVALID_ARG, "graph is NULL");
  for (int q = 0; q < ncodes; ++q) {
    const int nt = sh.stream_threads[q];
    if (nt != 0 && (nt < 64 || nt > 1024 || nt % 64))
      return set_error(LDPC_ERR_INVALID_ARG, "stream_threads must be 0 or a multiple of 64 in 64..1024");
    if (sh.split_slices[q] < 0) return set_error(LDPC_ERR_INVALID_ARG, "negative split_slices");
  }
  // codes decoded by the stream form: requested ones must fit, AUTO takes those that do
  uint32_t mask = 0;
  for (int q = 0; q < ncodes; ++q) {
    if (!((sh.stream_codes >> q) & 1u)) continue;
    const ldpc_status st = stream_ready_for(graphs[q], sh.stream_threads[q]);
    if (st == LDPC_OK)
      mask |= 1u << q;
    else if (sh.stream_codes != LDPC_STREAM_AUTO || st != LDPC_ERR_UNSUPPORTED)
      return st;
  }
  sh.stream_codes = mask;
  // codes decoded by the split form: requested ones, or AUTO: few tiles for the GPU
  uint32_t smask = 0;
  if (sh.split_codes) {
    int dev = 0, cus = 0;
    LDPC_HIP_CHECK(hipGetDevice(&dev));
    LDPC_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    for (int q = 0; q < ncodes; ++q) {
      if (!((sh.split_codes >> q) & 1u) || ((mask >> q) & 1u) || jobs[q].batch <= 0) continue;
      const long tiles = (jobs[q].batch + TW - 1) / TW;
      if (sh.split_codes != LDPC_SPLIT_AUTO || 2 * tiles < cus) smask |= 1u << q;
    }
  }
  sh.split_codes = smask;
  mask |= smask;  // from here on: codes decoded outside the persistent launch
  for (int q = 0; q < ncodes; ++q)
    if ((mask >> q) & 1u) sh.slots[q] = 0;
  if (sh.waves == 0) {
    // small batches (fewer 64-word tiles than compute units) get the widest workgroups
    int dev = 0, cus = 0;
    LDPC_HIP_CHECK(hipGetDevice(&dev));
    LDPC_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    long tiles = 0;
    for (int q = 0; q < ncodes; ++q)
      if (!((mask >> q) & 1u)) tiles += (jobs[q].batch + TW - 1) / TW;
    sh.waves = tiles < cus ? 16 : 8;
  }
  if (sh.waves < 1 || sh.waves > 16) return set_error(LDPC_ERR_INVALID_ARG, "waves must be in 1..16");
  if (sh.refill == 0) sh.refill = 1;
  if (sh.refill < 1 || sh.refill > kTile) return set_error(LDPC_ERR_INVALID_ARG, "refill must be in 1..64");
  if (sh.lanes < 0 || sh.lanes > kTile) return set_error(LDPC_ERR_INVALID_ARG, "lanes must be in 0..64");
  for (int q = 0; q < ncodes; ++q) {
    if (jobs[q].batch < 0 || jobs[q].max_iters < 0) return set_error(LDPC_ERR_INVALID_ARG, "negative batch/max_iters");
    if (sh.slots[q] < 0) return set_error(LDPC_ERR_INVALID_ARG, "negative slot count");
  }
  // automatic slot counts: fill the resident capacity, shared in proportion to words x edges
  bool need_auto = sh.lanes == 0;
  for (int q = 0; q < ncodes; ++q) need_auto |= sh.slots[q] == 0 && jobs[q].batch > 0 && !((mask >> q) & 1u);
  if (need_auto) {
    int dev = 0, cus = 0;
    LDPC_HIP_CHECK(hipGetDevice(&dev));
    LDPC_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    MultiArgs probe{};
    probe.njobs = ncodes;
    for (int q = 0; q < ncodes; ++q) {
      probe.jobs[q].kind = kernel_kind(graphs[q]);
      probe.jobs[q].dc_max = graphs[q]->dc_max;
      probe.jobs[q].nslots = jobs[q].batch > 0 && !((mask >> q) & 1u) ? 1 : 0;
    }
    int per_cu = 0;
    LDPC_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)multi_kernel_for(probe),
                                                                64 * sh.waves, 0));
    const double cap = (double)cus * (per_cu > 0 ? per_cu : 1);
    double total = 0;
    long words = 0;
    for (int q = 0; q < ncodes; ++q)
      if (!((mask >> q) & 1u)) {
        total += (double)jobs[q].batch * (double)graphs[q]->nnz;
        words += jobs[q].batch;
      }
    if (sh.lanes == 0) {
      // fewer words than 64 per resident slot: narrower slots spread them over more
      // compute units (a slot's iteration costs about the same with fewer busy lanes)
      const long per = (long)std::ceil((double)words / cap);
      sh.lanes = per >= TW ? TW : std::max(8, (int)((per + 7) / 8 * 8));
    }
    for (int q = 0; q < ncodes; ++q) {
      if (sh.slots[q] != 0 || jobs[q].batch == 0 || ((mask >> q) & 1u)) continue;
      const int peers = (jobs[q].batch + sh.lanes - 1) / sh.lanes;
      int s = total > 0 ? (int)(cap * (double)jobs[q].batch * (double)graphs[q]->nnz / total + 0.5) : 1;
      sh.slots[q] = std::max(1, std::min(s, peers));
    }
  }
  size_t bytes = 512;  // counters of the persistent launch, then of the stream-form codes
  for (int q = 0; q < ncodes; ++q) {
    if (jobs[q].batch == 0) sh.slots[q] = 0;
    bytes += (size_t)sh.slots[q] * tile_bytes(graphs[q]->nnz, graphs[q]->n);
  }
  for (int q = 0; q < ncodes; ++q)  // then one region per split-form code
    if ((smask >> q) & 1u) bytes += align256(split_workspace_bytes(graphs[q], jobs[q].batch));
  if (shape_out) *shape_out = sh;
  if (ws_bytes) *ws_bytes = bytes;
  return LDPC_OK;
}

ldpc_status multi_args(const ldpc_graph_t *graphs, int32_t ncodes, const ldpc_job *jobs, const int32_t *const *orders,
                       const ldpc_multi_shape &sh, void *ws, MultiArgs *a, int **counters, int *grid) {
  char *p = (char *)ws;
  *counters = (int *)p;
  p += 512;
  a->njobs = ncodes;
  a->refill_min = std::min(sh.refill, sh.lanes > 0 ? sh.lanes : kTile);
  a->lanes = sh.lanes > 0 ? sh.lanes : kTile;
  int slot = 0;
  for (int q = 0; q < ncodes; ++q) {
    MultiJob &J = a->jobs[q];
    const ldpc_job &j = jobs[q];
    if (j.batch > 0 && (!j.llr || !j.hard_bits || !j.posterior || !j.iters_used))
      return set_error(LDPC_ERR_INVALID_ARG, "NULL buffer in job " + std::to_string(q));
    J.g = graph_dev(graphs[q]);
    J.llr = j.llr;
    J.hard = j.hard_bits;
    J.post = j.posterior;
    J.iters = j.iters_used;
    J.batch = j.batch;
    J.max_iters = j.max_iters;
    J.slot0 = slot;
    J.nslots = sh.slots[q];
    J.kind = kernel_kind(graphs[q]);
    J.dc_max = graphs[q]->dc_max;
    J.ws = p;
    J.order = orders ? orders[q] : nullptr;
    p += (size_t)sh.slots[q] * tile_bytes(graphs[q]->nnz, graphs[q]->n);
    slot += sh.slots[q];
  }
  *grid = slot;
  return LDPC_OK;
}

namespace {
constexpr int kSideDevices = 64;
}  // namespace

// Side streams are created on first use, one per device and host thread, and kept for
// the process.
ldpc_status multi_side_stream(SideStream **out) {
  thread_local SideStream cache[kSideDevices];
  *out = nullptr;
  int dev = 0;
  LDPC_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kSideDevices) return LDPC_OK;  // no side stream: everything on the caller's
  SideStream &c = cache[dev];
  if (!c.s) {
    LDPC_HIP_CHECK(hipStreamCreateWithFlags(&c.s, hipStreamNonBlocking));
    LDPC_HIP_CHECK(hipEventCreateWithFlags(&c.fork, hipEventDisableTiming));
    LDPC_HIP_CHECK(hipEventCreateWithFlags(&c.join, hipEventDisableTiming));
  }
  *out = &c;
  return LDPC_OK;
}

ldpc_status multi_enqueue(const MultiArgs &a, int *counters, int grid, int waves, int early_stop,
                          hipStream_t stream, const StreamCodes *sc, const SplitCodes *sp) {
  SideStream *side = nullptr;
  if (sp && sp->n > 0 && ((sc && sc->n > 0) || grid > 0)) {
    ldpc_status st = multi_side_stream(&side);
    if (st != LDPC_OK) return st;
  }
  hipStream_t split_stream = stream;
  if (side) {
    LDPC_HIP_CHECK(hipEventRecord(side->fork, stream));
    LDPC_HIP_CHECK(hipStreamWaitEvent(side->s, side->fork, 0));
    split_stream = side->s;
  }
  if (sp) {
    for (int i = 0; i < sp->n; ++i) {
      const ldpc_job &j = sp->job[i];
      ldpc_status st = launch_split_decode(sp->g[i], j.llr, false, j.batch, j.max_iters, early_stop, j.hard_bits,
                                           j.posterior, j.iters_used, sp->ws[i], sp->slices[i], split_stream);
      if (st != LDPC_OK) return st;
    }
  }
  if (side) LDPC_HIP_CHECK(hipEventRecord(side->join, side->s));
  if (sc) {
    for (int i = 0; i < sc->n; ++i) {
      const ldpc_job &j = sc->job[i];
      ldpc_status st = launch_stream_decode(sc->g[i], j.llr, false, j.batch, j.max_iters, early_stop, j.hard_bits,
                                            j.posterior, j.iters_used, counters + 64 + sc->code[i], sc->threads[i],
                                            stream);
      if (st != LDPC_OK) return st;
    }
  }
  hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, stream, counters, a.njobs);
  LDPC_HIP_CHECK(hipGetLastError());
  if (grid > 0) {
    hipLaunchKernelGGL(multi_kernel_for(a), dim3(grid), dim3(64 * waves), 0, stream, a, counters,
                       (int)(early_stop != 0));
    LDPC_HIP_CHECK(hipGetLastError());
  }
  if (side) LDPC_HIP_CHECK(hipStreamWaitEvent(stream, side->join, 0));
  return LDPC_OK;
}
