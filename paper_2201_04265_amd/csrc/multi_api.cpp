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
    sc->threads[sc->n] = sh.stream_threads[q];
    ++sc->n;
  }
  // split-form regions follow the slot states (the layout of multi_resolve's size)
  size_t off = 512;
  for (int q = 0; q < ncodes; ++q) off += slot_region_bytes(graphs[q], sh, q);
  sp->n = 0;
  for (int q = 0; q < ncodes; ++q) {
    if (!((sh.split_codes >> q) & 1u)) continue;
    const ldpc_job &j = jobs[q];
    if (!j.llr || !j.hard_bits || !j.posterior || !j.iters_used)
      return set_error(LDPC_ERR_INVALID_ARG, "NULL buffer in job " + std::to_string(q));
    sp->g[sp->n] = graphs[q];
    sp->job[sp->n] = j;
    sp->ws[sp->n] = (char *)ws + off;
    sp->slices[sp->n] = sh.split_slices[q];
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

namespace {

// Times one shape: a warm-up run, then timed runs of the whole batched call, as many as
// fit in about 40 ms (2 to 16), and returns their median: short batches (a few ms) are
// otherwise decided by launch-to-launch noise.
struct Timer {
  const ldpc_graph_t *graphs;
  int32_t ncodes;
  const ldpc_job *jobs;
  const int32_t *const *orders;
  int32_t early_stop;
  hipStream_t stream;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  hipEvent_t t0 = nullptr, t1 = nullptr;

  ldpc_status run_once(const ldpc_multi_shape &c, float *ms) {
    LDPC_HIP_CHECK(hipEventRecord(t0, stream));
    ldpc_status st = ldpc_decode_multi(graphs, ncodes, jobs, orders, early_stop, &c, ws, ws_bytes, stream);
    if (st != LDPC_OK) return st;
    LDPC_HIP_CHECK(hipEventRecord(t1, stream));
    LDPC_HIP_CHECK(hipEventSynchronize(t1));
    LDPC_HIP_CHECK(hipEventElapsedTime(ms, t0, t1));
    return LDPC_OK;
  }

  ldpc_status time(const ldpc_multi_shape &c, float *ms_out) {
    size_t need = 0;
    ldpc_status st = multi_resolve(graphs, ncodes, jobs, &c, nullptr, &need);
    if (st != LDPC_OK) return st;
    if (need > ws_bytes) {  // grow the temporary workspace
      if (ws) (void)hipFree(ws);
      ws = nullptr;
      ws_bytes = 0;
      if (hipMalloc(&ws, need) != hipSuccess) return set_error(LDPC_ERR_OUT_OF_MEMORY, "autotune workspace");
      ws_bytes = need;
    }
    float warm = 0;
    if ((st = run_once(c, &warm)) != LDPC_OK) return st;
    const int reps = std::max(2, std::min(16, (int)(40.0f / std::max(warm, 0.01f))));
    std::vector<float> t((size_t)reps);
    for (int r = 0; r < reps; ++r)
      if ((st = run_once(c, &t[(size_t)r])) != LDPC_OK) return st;
    std::sort(t.begin(), t.end());
    *ms_out = reps % 2 ? t[(size_t)reps / 2] : 0.5f * (t[(size_t)reps / 2 - 1] + t[(size_t)reps / 2]);
    return LDPC_OK;
  }
};

}  // namespace

extern "C" ldpc_status ldpc_autotune_multi(const ldpc_graph_t *graphs, int32_t ncodes, const ldpc_job *jobs,
                                           const int32_t *const *orders, int32_t early_stop, uint32_t flags,
                                           hipStream_t stream, ldpc_multi_shape *best, float *best_ms) {
  if (!best) return set_error(LDPC_ERR_INVALID_ARG, "best is NULL");
  if (flags & ~LDPC_TUNE_PERSISTENT_ONLY) return set_error(LDPC_ERR_INVALID_ARG, "unknown flag");
  const bool forms = !(flags & LDPC_TUNE_PERSISTENT_ONLY);
  ldpc_multi_shape base{};
  base.stream_codes = forms ? LDPC_STREAM_AUTO : 0u;
  base.split_codes = forms ? LDPC_SPLIT_AUTO : 0u;
  ldpc_multi_shape cur{};
  ldpc_status st = multi_resolve(graphs, ncodes, jobs, &base, &cur, nullptr);
  if (st != LDPC_OK) return st;
  // which codes may take the stream form at all
  uint32_t can_stream = 0;
  for (int q = 0; q < ncodes; ++q)
    if (jobs[q].batch > 0 && stream_ready_for(graphs[q], 0) == LDPC_OK) can_stream |= 1u << q;
  Timer T{graphs, ncodes, jobs, orders, early_stop, stream};
  LDPC_HIP_CHECK(hipEventCreate(&T.t0));
  LDPC_HIP_CHECK(hipEventCreate(&T.t1));
  float cur_ms = 0;
  // a candidate is given with explicit forms and automatic persistent slots
  auto with_forms = [&](uint32_t smask, uint32_t pmask) {
    ldpc_multi_shape c = cur;
    c.stream_codes = smask;
    c.split_codes = pmask;
    for (int q = 0; q < ncodes; ++q) c.slots[q] = 0;
    c.lanes = 0;
    c.waves = 0;
    return c;
  };
  auto attempt = [&](const ldpc_multi_shape &c) -> ldpc_status {
    // shapes the launch cannot take (group slots beyond the resident capacity) are skipped
    if (multi_resolve(graphs, ncodes, jobs, &c, nullptr, nullptr) != LDPC_OK) return LDPC_OK;
    float ms = 0;
    ldpc_status s2 = T.time(c, &ms);
    if (s2 != LDPC_OK) return s2;
    if (ms < cur_ms) {
      cur_ms = ms;
      cur = c;
    }
    return LDPC_OK;
  };
  st = T.time(cur, &cur_ms);
  const ldpc_multi_shape start_shape = cur;
  // 1. the form of each code, one code at a time
  for (int q = 0; q < ncodes && st == LDPC_OK && forms; ++q) {
    if (jobs[q].batch == 0) continue;
    const uint32_t bit = 1u << q;
    const uint32_t sm = cur.stream_codes & ~bit, pm = cur.split_codes & ~bit;
    if ((can_stream & bit) && !(cur.stream_codes & bit)) st = attempt(with_forms(sm | bit, pm));
    if (st == LDPC_OK && !(cur.split_codes & bit) && !(cur.stream_codes & bit)) st = attempt(with_forms(sm, pm | bit));
    if (st == LDPC_OK && ((cur.stream_codes | cur.split_codes) & bit)) st = attempt(with_forms(sm, pm));
  }
  // 2. workgroup sizes of the stream-form codes, slices of the split-form codes
  for (int q = 0; q < ncodes && st == LDPC_OK; ++q) {
    if (jobs[q].batch == 0) continue;
    if ((cur.stream_codes >> q) & 1u) {
      for (int nt : {256, 512, 1024}) {
        ldpc_multi_shape c = cur;
        c.stream_threads[q] = nt;
        if (stream_ready_for(graphs[q], nt) != LDPC_OK) continue;
        if ((st = attempt(c)) != LDPC_OK) break;
      }
    } else if ((cur.split_codes >> q) & 1u) {
      for (int sl : {4, 16, 64}) {
        ldpc_multi_shape c = cur;
        c.split_slices[q] = sl;
        if ((st = attempt(c)) != LDPC_OK) break;
      }
    }
  }
  // 3. the persistent launch's shape, when some code uses it
  bool persistent = false;
  for (int q = 0; q < ncodes; ++q) persistent |= cur.slots[q] > 0 || (jobs[q].batch > 0 &&
                                                  !(((cur.stream_codes | cur.split_codes) >> q) & 1u));
  if (persistent && st == LDPC_OK) {
    const ldpc_multi_shape start = cur;
    for (int waves : {8, 16}) {
      for (int lanes : {64, 32, 16}) {
        ldpc_multi_shape b0 = start;
        b0.waves = waves;
        b0.lanes = lanes;
        for (int q = 0; q < ncodes; ++q) b0.slots[q] = b0.span[q] = 0;
        ldpc_multi_shape autos{};
        if ((st = multi_resolve(graphs, ncodes, jobs, &b0, &autos, nullptr)) != LDPC_OK) break;
        bool groups = false;
        for (int q = 0; q < ncodes; ++q) groups |= autos.span[q] > 1;
        // slot counts scaled around the automatic ones (automatic spans kept)
        for (double scale : {0.5, 1.0, 2.0}) {
          for (int refill : {1, 4}) {
            ldpc_multi_shape c = autos;
            c.refill = refill;
            for (int q = 0; q < ncodes; ++q) {
              const int per = (jobs[q].batch + autos.lanes - 1) / std::max(1, autos.lanes);
              c.slots[q] = autos.slots[q] ? std::max(1, std::min(per, (int)(autos.slots[q] * scale + 0.5))) : 0;
            }
            if ((st = attempt(c)) != LDPC_OK) break;
          }
          if (st != LDPC_OK) break;
        }
        // group slots: half and a quarter of the automatic spans, and none
        for (int div : {2, 4, 0}) {
          if (!groups || st != LDPC_OK) break;
          ldpc_multi_shape c = autos;
          for (int q = 0; q < ncodes; ++q)
            if (autos.span[q] > 1) c.span[q] = div ? std::max(1, autos.span[q] / div) : 1;
          st = attempt(c);
        }
        if (st != LDPC_OK) break;
      }
      if (st != LDPC_OK) break;
    }
    // 4. each code's span, doubled or halved, one code at a time (from the best so far:
    // codes differ in iterations per word, which the automatic share does not know)
    for (int q = 0; q < ncodes && st == LDPC_OK; ++q) {
      if (cur.slots[q] <= 0) continue;
      const int base_span = std::max(1, cur.span[q]);
      for (int sp : {2 * base_span, base_span / 2}) {
        if (sp < 1 || sp > kMaxSpan || sp == base_span) continue;
        ldpc_multi_shape c = cur;
        c.span[q] = sp;
        if ((st = attempt(c)) != LDPC_OK) break;
      }
    }
  }
  // 5. the winner against the automatic start, timed again side by side: a search decided by
  // one noisy measurement must not return a shape slower than the heuristics, so the start
  // stays unless the winner is faster by more than the timing noise (2 %)
  if (st == LDPC_OK) {
    float again = 0, start_again = 0;
    st = T.time(cur, &again);
    if (st == LDPC_OK) st = T.time(start_shape, &start_again);
    if (st == LDPC_OK && start_again <= again * 1.02f) {
      cur = start_shape;
      cur_ms = start_again;
    } else if (st == LDPC_OK) {
      cur_ms = again;
    }
  }
  (void)hipEventDestroy(T.t0);
  (void)hipEventDestroy(T.t1);
  if (T.ws) (void)hipFree(T.ws);
  if (st != LDPC_OK) return st;
  *best = cur;
  if (best_ms) *best_ms = cur_ms;
  return LDPC_OK;
}
