// Batched persistent decoder: several codes, one launch, per-word refill.
//
// Sec. III-C distributes a batch of whole words over workers that decode them
// one after another.  Here a worker is a "slot": the state of 64 words (one per
// lane) of a single code, with the same tile layout and the same check / variable
// updates as the plain decoder, served by one workgroup or by a group of `span`
// workgroups that share the slot's checks and variables.  A lane whose word stops
// (zero syndrome or max_iters) writes that word's outputs and claims the next word
// of its code from a per-code atomic counter (one atomic per slot per refill), so
// no lane waits for the slowest word of a tile.  All codes of a batch run in one
// launch.  Per word the arithmetic and its order are those of the plain decoder,
// so outputs are bit-identical to it whatever lane, slot or group ran the word.
//
// Step G of a slot: check phase writes E into E[(G+1)&1] and tests the syndrome of
// the decisions the messages carry; lanes that stop at G have their last messages in
// E[G&1] (all lanes of a slot share the step parity, so buffer choice is uniform).
// The variable pass of the step then serves three kinds of lanes at once: running
// lanes update their messages, lanes whose word stopped write its posterior (from
// their own E buffer) and decisions out, and lanes that took a new word load its
// LLRs and derive its first messages -- one pass over the variables instead of
// separate output, input and update passes.
//
// A group slot (span > 1) is the answer to batches with few words of a long code:
// one workgroup per 64 words would leave most compute units idle for the whole
// decode.  Its workgroups split every phase (check c and variable v go to the
// group's wavefront c and v mod span x waves) and meet at a barrier of the group
// where a single workgroup meets __syncthreads: after the check phase (with the
// lanes' unsatisfied-check masks OR-ed in global memory), after a refill's word
// claims, and at the end of each step.  Every member keeps the same per-lane state
// (the same masks give the same decisions), so all members take the same branches
// and meet at the same barriers.
#include <cmath>
#include <cstdlib>

#include "internal.h"
#include "multi.h"
#include "tile.h"

namespace ldpc {

// Barrier of the `span` workgroups of a group slot.  The members may sit on different
// XCDs, whose L2 caches are not coherent with each other, so what a member stored must be
// written back to memory before the others read it, and their caches must drop stale
// copies: every wavefront waits for its own stores to complete, the workgroup meets,
// then one thread writes the L2 back (agent-scope release: the write-back covers every
// completed store in that L2, whichever wavefront made it), arrives on the slot's counter,
// waits for the other members and invalidates its caches (agent-scope acquire: the
// compute unit's L1 and the L2 copies, for every wavefront of the workgroup, which meets
// again before reading).  One write-back and one invalidation per workgroup and barrier,
// not one per wavefront.
// The host launches group slots only when every workgroup of the launch can be resident
// at once, so the wait ends.  It is bounded all the same: after `limit` polls, or as soon
// as the launch's fault word is set, the barrier fails -- it sets the fault word, and the
// whole workgroup leaves its slot; the other members' waits then fail too, so the launch
// ends with the fault word telling the caller that its outputs are invalid.
constexpr unsigned kSpinLimit = 1u << 21;  // polls of about a microsecond each

__device__ __forceinline__ bool group_barrier(int *cnt, int span, int &epoch, int *fault, unsigned limit,
                                              int *fail_lds) {
  __builtin_amdgcn_s_waitcnt(0);  // this wavefront's loads and stores are complete
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const int target = (epoch + 1) * span;
    __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int failed = 0;
    for (unsigned spins = 0; __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target; ++spins) {
      if (spins >= limit || __hip_atomic_load(fault, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        __hip_atomic_fetch_or(fault, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        failed = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *fail_lds = failed;
  }
  __syncthreads();
  ++epoch;
  return *fail_lds == 0;
}

__device__ __forceinline__ int next_word(const MultiJob &J, int w) {
  return w < J.batch ? (J.order ? J.order[w] : w) : -1;
}

// The variable pass of a step (one slot; wavefront gw of GW takes variable groups gw, gw + GW,
// ... of VB consecutive variables each):
//   running: Eq. 7 posterior and Eq. 6 messages from this step's E (En), as var_update;
//   out:     the lane's stopped word `out_word` gets the posterior of its last iteration,
//            recomputed from its own E buffer (E1 if out_odd, else E0) with the same
//            summation -- or R itself if it stopped before any iteration -- and its
//            decisions, straight into the word's row of [B][n];
//   fresh:   the lane took word `new_word` (after writing out its old one): its LLRs go
//            to R and its first messages M = clamp(R) carry the channel decisions.
// The rows of [B][n] differ per lane, so each such access touches its own cache line; with
// VB = 4 (VB must divide n) a lane moves four variables of its row per access (16-byte
// posterior and LLR accesses, 4-byte decision stores) instead of one.  Idle lanes load nothing.
template <int DV, int VB>
__device__ __forceinline__ void slot_pass(const MultiJob &J, TileState st, const float *En, bool running, bool out,
                                          bool out_odd, int out_word, int out_it, bool fresh, int new_word, int gw,
                                          int GW, int lane) {
  constexpr int DMAX = DV > 0 ? DV : -DV;
  static_assert(VB == 1 || VB == 4, "variables per group");
  if (!(running || out || fresh)) return;
  const GraphDev &g = J.g;
  // a stopped word's last messages are in the other buffer: reading them costs this
  // pass an extra cache line per load, which is cheaper than writing every lane's
  // posterior each step or making the lane skip a check phase (whose masked stores
  // would leave partly written lines for the next reads to merge)
  const float *Eb = out ? (out_odd ? st.E1 : st.E0) : En;
  const size_t n = (size_t)g.n;
  float *prow = J.post + (out ? (size_t)out_word * n : 0);
  uint8_t *hrow = J.hard + (out ? (size_t)out_word * n : 0);
  const float *src = J.llr + (fresh ? (size_t)new_word * n : 0);
  const int groups = g.n / VB;
  for (int qv = gw; qv < groups; qv += GW) {
    const int v0 = qv * VB;
    float x[VB], lo[VB];
    if (fresh) {
      if constexpr (VB == 4) {
        const float4 f = *reinterpret_cast<const float4 *>(src + v0);
        x[0] = f.x;
        x[1] = f.y;
        x[2] = f.z;
        x[3] = f.w;
      } else {
        x[0] = src[v0];
      }
    }
#pragma unroll
    for (int i = 0; i < VB; ++i) {
      const int v = v0 + i;
      int p0, dv;
      var_range<DV>(g, v, p0, dv);
      float ev[DMAX];
      int eid[DMAX];
      const float r = st.R[v * TW + lane];
      const double L = var_posterior<DV>(r, Eb, g.var_edges, p0, dv, lane, ev, eid);
      lo[i] = out_it > 0 ? (float)L : r;
      if (running) {
        const bool z = (float)L <= 0.0f;
#pragma unroll
        for (int j = 0; j < DMAX; ++j)
          if (DV > 0 || j < dv) st.M[eid[j] * TW + lane] = v2c_store(var_extrinsic(L, ev[j]), z);
      } else if (fresh) {
        st.R[v * TW + lane] = x[i];
        const float mx = v2c_store(x[i], x[i] <= 0.0f);
#pragma unroll
        for (int j = 0; j < DMAX; ++j)
          if (DV > 0 || j < dv) st.M[eid[j] * TW + lane] = mx;
      }
    }
    if (out) {
      if constexpr (VB == 4) {
        *reinterpret_cast<float4 *>(prow + v0) = make_float4(lo[0], lo[1], lo[2], lo[3]);
        const uint32_t h = (lo[0] <= 0.0f ? 1u : 0u) | (lo[1] <= 0.0f ? 1u << 8 : 0u) |
                           (lo[2] <= 0.0f ? 1u << 16 : 0u) | (lo[3] <= 0.0f ? 1u << 24 : 0u);
        *reinterpret_cast<uint32_t *>(hrow + v0) = h;
      } else {
        prow[v0] = lo[0];
        hrow[v0] = lo[0] <= 0.0f ? 1 : 0;
      }
    }
  }
}

// slot_pass with four variables per group where the degree is fixed and n allows it.
template <int DV>
__device__ __forceinline__ void slot_pass_any(const MultiJob &J, TileState st, const float *En, bool running, bool out,
                                              bool out_odd, int out_word, int out_it, bool fresh, int new_word,
                                              int gw, int GW, int lane) {
  if constexpr (DV > 0) {
    if ((J.g.n & 3) == 0) {
      slot_pass<DV, 4>(J, st, En, running, out, out_odd, out_word, out_it, fresh, new_word, gw, GW, lane);
      return;
    }
  }
  slot_pass<DV, 1>(J, st, En, running, out, out_odd, out_word, out_it, fresh, new_word, gw, GW, lane);
}

// One slot (member `member` of its `span` workgroups): lanes take words of job J until
// its queue is empty.  A lane whose word stops becomes pending; pending lanes are
// written out and refilled together once at least `refill_min` of them wait or no
// lane is running.  unsat_w and lane_lds are the workgroup's LDS scratch.
template <int DC, int DV>
__device__ void run_slot(const MultiJob &J, int local_slot, int member, int *counter, int *fault,
                         unsigned spin_limit, int early_stop, int refill_min, int lanes, unsigned long long *unsat_w,
                         int *lane_lds, int *fail_lds, int wave, int W, int lane, float *psl) {
  const GraphDev &g = J.g;
  const TileState st = tile_state_block(J.ws + (size_t)local_slot * tile_bytes(g.nnz, g.n), g.nnz, g.n);
  const int span = J.span;
  const bool group = span > 1;
  int *sync = group ? J.sync + (size_t)local_slot * kSyncInts : nullptr;
  int epoch = 0;
  const int gw = member * W + wave, GW = span * W;
  int *lw = group ? sync + kSyncLaneWords : lane_lds;  // lane -> word table of the slot
  // A failed group barrier (see group_barrier) clears `ok`; the workgroup then stops waiting at
  // the slot's barriers, finishes the step (its outputs are invalid anyway) and leaves.
  bool ok = true;
  auto slot_barrier = [&]() {
    if (!group)
      __syncthreads();
    else if (ok)
      ok = group_barrier(sync, span, epoch, fault, spin_limit, fail_lds);
  };

  if (member == 0 && wave == 0) {  // lanes >= `lanes` never take a word
    int base = 0;
    if (lane == 0) base = atomicAdd(counter, lanes);
    base = __shfl(base, 0);
    lw[lane] = lane < lanes ? next_word(J, base + lane) : -1;
  }
  slot_barrier();
  int word = lw[lane];
  bool has = word >= 0;  // lane holds a word (running or pending)
  bool pending = false;  // its word has stopped and waits for output
  bool odd = false;      // its last messages are in E1 (else E0)
  int it_lane = 0;
  if (!ok || __ballot(has) == 0ull) return;  // same in every member: nothing left for this slot
  slot_pass_any<DV>(J, st, st.E0, false, false, false, 0, 0, has, word, gw, GW, lane);
  slot_barrier();

  for (int G = 0;; ++G) {
    float *En = ((G + 1) & 1) ? st.E1 : st.E0;
    const bool active = has && !pending;
    int unsat = 0;
    if (active) {  // idle and stopped lanes load nothing
      for (int c = gw; c < g.m; c += GW) {
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
    if (group) {  // the members' masks meet in global memory (two, by step parity)
      unsigned long long *mk = (unsigned long long *)(sync + kSyncMasks);
      if (threadIdx.x == 0 && um) __hip_atomic_fetch_or(mk + (G & 1), um, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      slot_barrier();
      um = __hip_atomic_load(mk + (G & 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // the other parity's mask was last read in step G-1, before this barrier; cleared
      // here, the clear is visible to every member after the barrier that ends this step
      if (member == 0 && threadIdx.x == 0) mk[(G + 1) & 1] = 0ull;
    }
    const bool lane_unsat = (um >> lane) & 1ull;
    const bool stop = active && ((early_stop && !lane_unsat) || it_lane == J.max_iters);
    if (stop) odd = (G & 1) != 0;  // E^(it) was written at step G-1 into E[G & 1]
    pending = pending || stop;
    const bool running = active && !stop;
    const unsigned long long pmask = __ballot(pending);
    const unsigned long long rmask = __ballot(running);
    bool out = false, fresh = false;
    const int out_word = word, out_it = it_lane;
    if (pmask != 0ull && (__popcll(pmask) >= refill_min || rmask == 0ull)) {  // same in every wave and member
      if (member == 0 && wave == 0) {
        if (pending) J.iters[word] = it_lane;
        int base = 0;
        if (lane == 0) base = atomicAdd(counter, __popcll(pmask));
        base = __shfl(base, 0);
        const int rank = __popcll(pmask & ((1ull << lane) - 1ull));
        lw[lane] = pending ? next_word(J, base + rank) : word;
      }
      slot_barrier();
      const int nw = lw[lane];
      out = pending;
      fresh = pending && nw >= 0;
      if (pending) {
        word = nw;
        has = nw >= 0;
        it_lane = 0;
        pending = false;
      }
    }
    slot_pass_any<DV>(J, st, En, running, out, odd, out_word, out_it, fresh, word, gw, GW, lane);
    if (!ok || __ballot(has) == 0ull) break;  // same value in every wave and member
    if (running) ++it_lane;
    slot_barrier();
  }
}

// Workgroup -> job: job q owns workgroups [wg0, wg0 + nslots x span); within them
// workgroup wg0 + k x nslots + s is member k of slot s.
__device__ __forceinline__ int find_job(const MultiArgs &a, int wg) {
  int q = 0;
  for (int i = 0; i < a.njobs; ++i)
    if (wg >= a.jobs[i].wg0) q = i;
  return q;
}

template <int DC, int DV>
__device__ __forceinline__ void run_workgroup(const MultiArgs &a, int *counters, int early_stop, float *psl) {
  __shared__ unsigned long long unsat_w[16];
  __shared__ int lane_lds[TW];
  __shared__ int fail_lds;
  const int q = find_job(a, blockIdx.x);
  const MultiJob &J = a.jobs[q];
  const int local = (int)blockIdx.x - J.wg0;
  run_slot<DC, DV>(J, local % J.nslots, local / J.nslots, counters + q, counters + kFaultInt,
                   a.spin_limit, early_stop, a.refill_min, a.lanes, unsat_w, lane_lds,
                   &fail_lds, wave_id(), blockDim.x >> 6, lane_id(), psl);
}

template <int DC, int DV>
__global__ void __launch_bounds__(1024) multi_kernel_single(MultiArgs a, int *counters, int early_stop) {
  constexpr int kPsl = check_psl_floats<DC>();  // LDS of high runtime degrees (check_update)
  __shared__ float psl_buf[kPsl > 0 ? 16 * kPsl : 1];
  run_workgroup<DC, DV>(a, counters, early_stop, kPsl > 0 ? psl_buf + wave_id() * kPsl : nullptr);
}

// Largest check degree of a degree specialisation (negative: runtime degrees up to -DC).
constexpr int kind_dc_bound(int dc) { return dc > 0 ? dc : -dc; }

// Codes of different degree profiles in one launch: each workgroup runs the instance
// compiled for its own code's degrees (a switch on the code's specialisation), with the
// generic runtime-degree path up to the batch's largest check degree -DC for the rest.
// One register allocation covers every instance, that of the most demanding one.
template <int DC>
__global__ void __launch_bounds__(1024) multi_kernel_mixed(MultiArgs a, int *counters, int early_stop) {
  constexpr int kPsl = check_psl_floats<DC>();  // LDS of high runtime degrees (check_update)
  __shared__ float psl_buf[kPsl > 0 ? 16 * kPsl : 1];
  float *psl = kPsl > 0 ? psl_buf + wave_id() * kPsl : nullptr;
  const int kind = a.jobs[find_job(a, blockIdx.x)].kind;
#define LDPC_RUN(C, V)                                              \
  if constexpr (kind_dc_bound(C) <= -DC)                            \
    run_workgroup<C, V>(a, counters, early_stop, psl);              \
  else                                                              \
    run_workgroup<DC, -LDPC_MAX_VAR_DEGREE>(a, counters, early_stop, psl)
  LDPC_KIND_SWITCH(kind, LDPC_RUN)
#undef LDPC_RUN
}

// Zeroes the per-code counters, the fault word and the group slots' barrier words.
__global__ void reset_multi(MultiArgs a, int *counters) {
  if (threadIdx.x < (unsigned)a.njobs) counters[threadIdx.x] = 0;
  if (threadIdx.x == 0) counters[kFaultInt] = 0;
  for (int q = 0; q < a.njobs; ++q) {
    const MultiJob &J = a.jobs[q];
    if (!J.sync) continue;
    const int n = J.nslots * kSyncInts;
    for (int i = threadIdx.x; i < n; i += blockDim.x) J.sync[i] = 0;
  }
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
  for (int q = 0; q < ncodes; ++q)
    if (sh.span[q] < 0 || sh.span[q] > kMaxSpan)
      return set_error(LDPC_ERR_INVALID_ARG, "span must be in 0.." + std::to_string(kMaxSpan));
  auto persistent = [&](int q) { return jobs[q].batch > 0 && !((mask >> q) & 1u); };
  // automatic slot counts: fill the resident capacity, shared in proportion to words x
  // edges; a code whose words fill fewer slots than its share gets group slots (span > 1)
  bool need_auto = sh.lanes == 0, any_group = false, any_persistent = false;
  for (int q = 0; q < ncodes; ++q) {
    if (!persistent(q)) continue;
    any_persistent = true;
    need_auto |= sh.slots[q] == 0 || sh.span[q] == 0;
    any_group |= sh.span[q] > 1;
  }
  double cap = 0;  // workgroups of this launch the GPU holds resident at once
  if (any_persistent) {
    int dev = 0, cus = 0;
    LDPC_HIP_CHECK(hipGetDevice(&dev));
    LDPC_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    MultiArgs probe{};
    probe.njobs = ncodes;
    for (int q = 0; q < ncodes; ++q) {
      probe.jobs[q].kind = kernel_kind(graphs[q]);
      probe.jobs[q].dc_max = graphs[q]->dc_max;
      probe.jobs[q].nslots = persistent(q) ? 1 : 0;
    }
    int per_cu = 0;
    LDPC_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)multi_kernel_for(probe),
                                                                64 * sh.waves, 0));
    cap = (double)cus * (per_cu > 0 ? per_cu : 1);
  }
  if (need_auto) {
    double total = 0;
    for (int q = 0; q < ncodes; ++q)
      if (persistent(q)) total += (double)jobs[q].batch * (double)graphs[q]->nnz;
    if (sh.lanes == 0) sh.lanes = TW;
    for (int q = 0; q < ncodes; ++q) {
      if (!persistent(q)) continue;
      const int peers = (jobs[q].batch + sh.lanes - 1) / sh.lanes;
      const double share = total > 0 ? cap * (double)jobs[q].batch * (double)graphs[q]->nnz / total : 1.0;
      if (sh.slots[q] == 0) sh.slots[q] = std::max(1, std::min((int)(share + 0.5), peers));
      if (sh.span[q] == 0) {
        sh.span[q] = std::max(1, std::min(kMaxSpan, (int)(share / sh.slots[q])));
        any_group |= sh.span[q] > 1;
      }
    }
  }
  long wgs = 0;
  for (int q = 0; q < ncodes; ++q) {
    if (!persistent(q)) {
      sh.slots[q] = 0;
      sh.span[q] = 0;
    } else if (sh.span[q] == 0) {
      sh.span[q] = 1;
    }
    // a code's slots beyond what the GPU holds resident at once would only start once
    // its first slots leave, which they do when its queue is empty: they are dropped
    if (persistent(q) && cap > 0)
      sh.slots[q] = std::max(1, std::min(sh.slots[q], (int)(cap / std::max(1, sh.span[q]))));
    wgs += (long)sh.slots[q] * sh.span[q];
  }
  if (any_group && wgs > (long)cap) {
    // a group slot's workgroups wait for each other: every workgroup of the launch must
    // be resident at once.  Automatic spans shrink to fit, explicit ones are an error.
    for (int q = 0; q < ncodes; ++q)
      if (persistent(q) && shape_in && shape_in->span[q] > 1)
        return set_error(LDPC_ERR_INVALID_ARG, "group slots need " + std::to_string(wgs) +
                                                   " resident workgroups, the GPU holds " +
                                                   std::to_string((long)cap) + " of this kernel");
    while (wgs > (long)cap) {
      int best = -1;
      for (int q = 0; q < ncodes; ++q)
        if (persistent(q) && sh.span[q] > 1 && (best < 0 || sh.span[q] > sh.span[best])) best = q;
      if (best < 0) break;
      --sh.span[best];
      wgs -= sh.slots[best];
    }
  }
  size_t bytes = 512;  // counters of the persistent launch, then of the stream-form codes
  for (int q = 0; q < ncodes; ++q) bytes += slot_region_bytes(graphs[q], sh, q);
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
  // polls before a group barrier gives up; LDPC_GROUP_SPIN_LIMIT overrides the default so
  // that tests can force the failure path (a small value makes the waits fail at once)
  a->spin_limit = kSpinLimit;
  if (const char *e = std::getenv("LDPC_GROUP_SPIN_LIMIT")) a->spin_limit = (uint32_t)std::strtoul(e, nullptr, 10);
  int wg = 0;
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
    J.wg0 = wg;
    J.nslots = sh.slots[q];
    J.span = sh.slots[q] > 0 ? std::max(1, sh.span[q]) : 1;
    J.kind = kernel_kind(graphs[q]);
    J.dc_max = graphs[q]->dc_max;
    J.ws = p;
    J.sync = J.span > 1 ? (int32_t *)(p + (size_t)sh.slots[q] * tile_bytes(graphs[q]->nnz, graphs[q]->n)) : nullptr;
    J.order = orders ? orders[q] : nullptr;
    p += slot_region_bytes(graphs[q], sh, q);
    wg += sh.slots[q] * J.span;
  }
  *grid = wg;
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
  hipLaunchKernelGGL(reset_multi, dim3(1), dim3(1024), 0, stream, a, counters);
  LDPC_HIP_CHECK(hipGetLastError());
  if (grid > 0) {
    hipLaunchKernelGGL(multi_kernel_for(a), dim3(grid), dim3(64 * waves), 0, stream, a, counters,
                       (int)(early_stop != 0));
    LDPC_HIP_CHECK(hipGetLastError());
  }
  if (side) LDPC_HIP_CHECK(hipStreamWaitEvent(stream, side->join, 0));
  return LDPC_OK;
}
