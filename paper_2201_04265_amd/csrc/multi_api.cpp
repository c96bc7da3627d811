// C ABI of the batched persistent form: direct launches, captured plans, autotuner.
#include <algorithm>
#include <vector>

#include "internal.h"
#include "multi.h"
#include "tile.h"

extern "C" ldpc_status ldpc_multi_resolve(const ldpc_graph_t *graphs, int32_t ncodes, const ldpc_job *jobs,
                                          const ldpc_multi_shape *shape, ldpc_multi_shape *resolved,
                                          size_t *ws_bytes) {
  return multi_resolve(graphs, ncodes, jobs, shape, resolved, ws_bytes);
}

static ldpc_status multi_prepare(const ldpc_graph_t *graphs, int32_t ncodes, const ldpc_job *jobs,
                                 const int32_t *const *orders, const ldpc_multi_shape *shape, void *ws,
                                 size_t ws_bytes, MultiArgs *a, int **counters, int *grid, int *waves,
                                 StreamCodes *sc, SplitCodes *sp) {
  ldpc_multi_shape sh;
  size_t need = 0;
  ldpc_status st = multi_resolve(graphs, ncodes, jobs, shape, &sh, &need);
  if (st != LDPC_OK) return st;
  if (!ws) return set_error(LDPC_ERR_INVALID_ARG, "workspace is NULL");
  if (((uintptr_t)ws & 255) != 0) return set_error(LDPC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < need) return set_error(LDPC_ERR_INVALID_ARG, "workspace too small");
  *waves = sh.waves;
  sc->n = 0;
  for (int q = 0; q < ncodes; ++q) {
    if (!((sh.stream_codes >> q) & 1u) || jobs[q].batch == 0) continue;
    const ldpc_job &j = jobs[q];
    if (!j.llr || !j.hard_bits || !j.posterior || !j.iters_used)
      return set_error(LDPC_ERR_INVALID_ARG, "NULL buffer in job " + std::to_string(q));
    sc->code[sc->n] = q;
    sc->g[sc->n] = graphs[q];
    sc->job[sc->n] = j;
    ++sc->n;
  }
  // split-form regions follow the slot states (the layout of multi_resolve's size)
  size_t off = 512;
  for (int q = 0; q < ncodes; ++q) off += (size_t)sh.slots[q] * ldpc::tile_bytes(graphs[q]->nnz, graphs[q]->n);
  sp->n = 0;
  for (int q = 0; q < ncodes; ++q) {
    if (!((sh.split_codes >> q) & 1u)) continue;
    const ldpc_job &j = jobs[q];
    if (!j.llr || !j.hard_bits || !j.posterior || !j.iters_used)
      return set_error(LDPC_ERR_INVALID_ARG, "NULL buffer in job " + std::to_string(q));
    sp->g[sp->n] = graphs[q];
    sp->job[sp->n] = j;
    sp->ws[sp->n] = (char *)ws + off;
    ++sp->n;
    off += align256(split_workspace_bytes(graphs[q], j.batch));
  }
  return multi_args(graphs, ncodes, jobs, orders, sh, ws, a, counters, grid);
}

extern "C" ldpc_status ldpc_decode_multi(const ldpc_graph_t *graphs, int32_t ncodes, const ldpc_job *jobs,
                                         const int32_t *const *orders, int32_t early_stop,
                                         const ldpc_multi_shape *shape, void *workspace, size_t ws_bytes,
                                         hipStream_t stream) {
  MultiArgs a{};
  StreamCodes sc;
  SplitCodes sp;
  int *counters = nullptr;
  int grid = 0, waves = 0;
  ldpc_status st = multi_prepare(graphs, ncodes, jobs, orders, shape, workspace, ws_bytes, &a, &counters, &grid,
                                 &waves, &sc, &sp);
  if (st != LDPC_OK) return st;
  return multi_enqueue(a, counters, grid, waves, early_stop, stream, &sc, &sp);
}

struct ldpc_plan_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" ldpc_status ldpc_plan_create_multi(const ldpc_graph_t *graphs, int32_t ncodes, const ldpc_job *jobs,
                                              const int32_t *const *orders, int32_t early_stop,
                                              const ldpc_multi_shape *shape, void *workspace, size_t ws_bytes,
                                              hipStream_t capture_stream, ldpc_plan_t *out) {
  if (!out) return set_error(LDPC_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!capture_stream) return set_error(LDPC_ERR_INVALID_ARG, "capture needs a non-default stream");
  MultiArgs a{};
  StreamCodes sc;
  SplitCodes sp;
  int *counters = nullptr;
  int grid = 0, waves = 0;
  ldpc_status st = multi_prepare(graphs, ncodes, jobs, orders, shape, workspace, ws_bytes, &a, &counters, &grid,
                                 &waves, &sc, &sp);
  if (st != LDPC_OK) return st;
  if (sp.n > 0) {  // create the side stream before the capture begins
    SideStream *side = nullptr;
    st = multi_side_stream(&side);
    if (st != LDPC_OK) return st;
  }
  ldpc_plan_s *p = new (std::nothrow) ldpc_plan_s();
  if (!p) return set_error(LDPC_ERR_OUT_OF_MEMORY, "plan allocation");
  hipError_t e = hipStreamBeginCapture(capture_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    delete p;
    return hip_error(e, "hipStreamBeginCapture");
  }
  st = multi_enqueue(a, counters, grid, waves, early_stop, capture_stream, &sc, &sp);
  e = hipStreamEndCapture(capture_stream, &p->graph);
  if (st != LDPC_OK || e != hipSuccess) {
    if (p->graph) (void)hipGraphDestroy(p->graph);
    delete p;
    return st != LDPC_OK ? st : hip_error(e, "hipStreamEndCapture");
  }
  e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(p->graph);
    delete p;
    return hip_error(e, "hipGraphInstantiate");
  }
  *out = p;
  return LDPC_OK;
}

extern "C" ldpc_status ldpc_plan_launch(ldpc_plan_t plan, hipStream_t stream) {
  if (!plan) return set_error(LDPC_ERR_INVALID_ARG, "plan is NULL");
  LDPC_HIP_CHECK(hipGraphLaunch(plan->exec, stream));
  return LDPC_OK;
}

extern "C" ldpc_status ldpc_plan_destroy(ldpc_plan_t plan) {
  if (!plan) return set_error(LDPC_ERR_INVALID_ARG, "plan is NULL");
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  delete plan;
  return LDPC_OK;
}

// Candidate shapes: waves per workgroup x a scale of the automatic slot counts x refill threshold.
extern "C" ldpc_status ldpc_autotune_multi(const ldpc_graph_t *graphs, int32_t ncodes, const ldpc_job *jobs,
                                           const int32_t *const *orders, int32_t early_stop, hipStream_t stream,
                                           ldpc_multi_shape *best, float *best_ms) {
  if (!best) return set_error(LDPC_ERR_INVALID_ARG, "best is NULL");
  std::vector<ldpc_multi_shape> cands;
  for (int waves : {8, 16}) {
    ldpc_multi_shape base{};
    base.waves = waves;
    ldpc_multi_shape autos{};
    ldpc_status st = multi_resolve(graphs, ncodes, jobs, &base, &autos, nullptr);
    if (st != LDPC_OK) return st;
    for (double scale : {0.5, 1.0, 2.0}) {
      for (int refill : {1, 4}) {
        ldpc_multi_shape c = autos;
        c.refill = refill;
        for (int q = 0; q < ncodes; ++q) {
          const int tiles = (jobs[q].batch + kTile - 1) / kTile;
          c.slots[q] = jobs[q].batch ? std::max(1, std::min(tiles, (int)(autos.slots[q] * scale + 0.5))) : 0;
        }
        bool dup = false;
        for (auto &o : cands)
          dup |= std::equal(o.slots, o.slots + ncodes, c.slots) && o.waves == c.waves && o.refill == c.refill;
        if (!dup) cands.push_back(c);
      }
    }
  }
  size_t need = 0;
  for (auto &c : cands) {
    size_t b = 0;
    ldpc_status st = multi_resolve(graphs, ncodes, jobs, &c, nullptr, &b);
    if (st != LDPC_OK) return st;
    need = std::max(need, b);
  }
  void *ws = nullptr;
  hipError_t e = hipMalloc(&ws, need);
  if (e != hipSuccess) return set_error(LDPC_ERR_OUT_OF_MEMORY, "autotune workspace");
  hipEvent_t t0, t1;
  (void)hipEventCreate(&t0);
  (void)hipEventCreate(&t1);
  float best_t = 1e30f;
  ldpc_status st = LDPC_OK;
  for (auto &c : cands) {
    float tsum = 0;
    for (int rep = 0; rep < 3 && st == LDPC_OK; ++rep) {
      (void)hipEventRecord(t0, stream);
      st = ldpc_decode_multi(graphs, ncodes, jobs, orders, early_stop, &c, ws, need, stream);
      (void)hipEventRecord(t1, stream);
      (void)hipEventSynchronize(t1);
      float ms = 0;
      (void)hipEventElapsedTime(&ms, t0, t1);
      if (rep > 0) tsum += ms;  // first run warms up
    }
    if (st != LDPC_OK) break;
    if (tsum / 2 < best_t) {
      best_t = tsum / 2;
      *best = c;
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  (void)hipFree(ws);
  if (st == LDPC_OK && best_ms) *best_ms = best_t;
  return st;
}
