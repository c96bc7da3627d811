// Batched persistent decoder: device job descriptors and host helpers.
#pragma once

#include "internal.h"
#include "tile.h"

// Ints per group slot (span > 1) in global memory: the barrier's arrival counter, two
// 64-bit unsatisfied-check masks (even / odd steps) and the lane -> word table.
constexpr int kSyncInts = 128;
constexpr int kSyncMasks = 2;       // offset of the two masks (8-byte aligned)
constexpr int kSyncLaneWords = 64;  // offset of the lane -> word table
// Largest number of workgroups per slot.
constexpr int kMaxSpan = 64;
// Index (in ints) of the launch's fault word in the counter block at the start of the
// workspace: nonzero after a launch iff a group slot's barrier wait gave up.
constexpr int kFaultInt = 120;
static_assert(kFaultInt * 4 == LDPC_MULTI_FAULT_OFFSET, "fault word offset");

// One code of a batched launch, passed by value in the kernel arguments.
struct MultiJob {
  GraphDev g;
  const float *llr;
  uint8_t *hard;
  float *post;
  int32_t *iters;
  const int32_t *order;  // optional word order (NULL: 0..batch-1)
  char *ws;              // nslots tile states of this code
  int32_t batch, max_iters;
  int32_t wg0, nslots;    // workgroups [wg0, wg0 + nslots x span) serve this code's slots
  int32_t span;           // workgroups per slot
  int32_t *sync;          // span > 1: nslots x kSyncInts ints (zeroed before the launch)
  int32_t kind;           // degree specialisation (KernelKind)
  int32_t dc_max;         // largest check degree
};

struct MultiArgs {
  MultiJob jobs[LDPC_MAX_CODES];
  int32_t njobs;
  int32_t refill_min;  // pending lanes that trigger a refill
  int32_t lanes;       // lanes of a slot that take words (the others stay idle)
  uint32_t spin_limit; // polls before a group barrier gives up
};

using MultiKernel = void (*)(MultiArgs, int *, int);
MultiKernel multi_kernel_for(const MultiArgs &a);

// Workspace bytes of code q's slots: their tile states, then (group slots) their barrier words.
inline size_t slot_region_bytes(const ldpc_graph_s *g, const ldpc_multi_shape &sh, int q) {
  const size_t tiles = (size_t)sh.slots[q] * ldpc::tile_bytes(g->nnz, g->n);
  return tiles + (sh.span[q] > 1 ? (size_t)sh.slots[q] * kSyncInts * sizeof(int32_t) : 0);
}

// Validates the jobs, fills automatic slot counts and returns the workspace size.
ldpc_status multi_resolve(const ldpc_graph_t *graphs, int32_t ncodes, const ldpc_job *jobs,
                          const ldpc_multi_shape *shape_in, ldpc_multi_shape *shape_out, size_t *ws_bytes);
// Lays the jobs out over the workspace.
ldpc_status multi_args(const ldpc_graph_t *graphs, int32_t ncodes, const ldpc_job *jobs, const int32_t *const *orders,
                       const ldpc_multi_shape &sh, void *ws, MultiArgs *a, int **counters, int *grid);
// Codes of a batched decode that run in the stream form (host side).
struct StreamCodes {
  int n = 0;
  int code[LDPC_MAX_CODES];
  ldpc_graph_s *g[LDPC_MAX_CODES];
  ldpc_job job[LDPC_MAX_CODES];
  int32_t threads[LDPC_MAX_CODES];  // workgroup size (0 = automatic)
};

// Codes of a batched decode that run in the split form (host side), each with its
// workspace region.
struct SplitCodes {
  int n = 0;
  ldpc_graph_s *g[LDPC_MAX_CODES];
  ldpc_job job[LDPC_MAX_CODES];
  void *ws[LDPC_MAX_CODES];
  int32_t slices[LDPC_MAX_CODES];  // workgroups per tile (0 = automatic)
};

// A second stream (default priority) and two events: the split-form decodes of a
// batched call run on it beside the call's other launches (they touch disjoint outputs
// and workspace regions), forked from and joined back into the caller's stream.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
// The calling thread's side stream for the current device (created on first use; NULL
// if none is available).
ldpc_status multi_side_stream(SideStream **out);

// Enqueues the split-form decodes (on the side stream, forked from and joined back into
// `stream`, when there are other launches to overlap), the stream-form decodes
// (counters at counters + 64 + code), the counter reset and the persistent launch.
ldpc_status multi_enqueue(const MultiArgs &a, int *counters, int grid, int waves, int early_stop,
                          hipStream_t stream, const StreamCodes *sc, const SplitCodes *sp);
