// Internal declarations shared by the host-side sources of the decoder library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <mutex>
#include <vector>

#include "../../include/ldpc.h"
#include "host_layout.h"

// Tanner graph: the host arrays (GraphHost) plus device copies.
struct ldpc_graph_s : GraphHost {
  int device = 0;
  int32_t *d_row_ptr = nullptr, *d_col_idx = nullptr, *d_var_ptr = nullptr, *d_var_edges = nullptr;
  int32_t *d_var_xoff = nullptr;  // stream form: LDS byte offsets of the edges (var_edges order)
  int64_t stream_x_floats = 0;     // stream form: floats of a word's message array in LDS
  int32_t *d_xslot = nullptr;      // stream form, runtime degrees: start | degree << 16 per check
                                   // slot, then the variable groups' order and edge offsets
  int32_t stream_slots = 0;        // check slots in d_xslot (a multiple of 64)
  // Launch facts of the stream form, filled once on its first call (stream.hip).
  std::mutex stream_mu;
  bool stream_ready = false;
  int stream_cus = 0;
  int stream_lds_limit = 0;                // bytes of LDS one workgroup may use
  int stream_per_cu[5] = {0, 0, 0, 0, 0};  // resident workgroups per CU with 64 << i threads
  int lds_limit = 0;                       // LDS bytes per workgroup (unrolled form), 0 = not queried
};

// Systematic encoder (encode.hip): the host reduction of H and its device map.
struct ldpc_encoder_s {
  int32_t n = 0, k = 0, rank = 0;
  int32_t kw = 0, kwp = 0, rank4 = 0;     // message chunks, row stride of A, rows of A (multiple of 4)
  std::vector<int32_t> info, pivots;      // message positions (ascending), pivot column of row r
  int device = 0, lds_limit = 0;
  uint64_t *d_A = nullptr;                // [rank4][kwp]: bit j of row r = message bit j enters parity r
  int32_t *d_colmap = nullptr;            // [n]: message index j, or -1 - r for the pivot of row r
};


// Device view passed to kernels by value.
struct GraphDev {
  const int32_t *row_ptr;
  const int32_t *col_idx;
  const int32_t *var_ptr;
  const int32_t *var_edges;
  const int32_t *var_xoff;  // stream form: LDS byte offsets of the edges (var_edges order)
  int32_t m, n, nnz;
  int32_t dc, dv;  // uniform degrees, or 0 when irregular
};

inline GraphDev graph_dev(const ldpc_graph_s *g) {
  GraphDev d;
  d.row_ptr = g->d_row_ptr;
  d.col_idx = g->d_col_idx;
  d.var_ptr = g->d_var_ptr;
  d.var_edges = g->d_var_edges;
  d.var_xoff = g->d_var_xoff;
  d.m = g->m;
  d.n = g->n;
  d.nnz = (int32_t)g->nnz;
  d.dc = g->dc_min == g->dc_max ? g->dc_max : 0;
  d.dv = g->dv_min == g->dv_max ? g->dv_max : 0;
  return d;
}

// Expands F(DC, DV) for the specialisation of `kind` (DC/DV < 0: generic up to -DC/-DV).
#define LDPC_KIND_SWITCH(kind, F)                         \
  switch (kind) {                                         \
    case KIND_6_3: F(6, 3); break;                        \
    case KIND_4_3: F(4, 3); break;                        \
    case KIND_12_3: F(12, 3); break;                      \
    case KIND_15_3: F(15, 3); break;                      \
    case KIND_12_6: F(12, 6); break;                      \
    case KIND_12_9: F(12, 9); break;                      \
    case KIND_G8: F(-8, -LDPC_MAX_VAR_DEGREE); break;     \
    case KIND_G16: F(-16, -LDPC_MAX_VAR_DEGREE); break;   \
    case KIND_G24: F(-24, -kG24MaxVarDegree); break;      \
    default: F(-LDPC_MAX_CHECK_DEGREE, -LDPC_MAX_VAR_DEGREE); break; \
  }

// Error reporting: thread-local detail of the last failure.
ldpc_status set_error(ldpc_status s, const std::string &msg);
ldpc_status hip_error(hipError_t e, const char *what);

#define LDPC_HIP_CHECK(call)                               \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return hip_error(e_, #call);     \
  } while (0)


inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Plain decode launcher (decode.hip).
ldpc_status launch_plain_decode(const ldpc_graph_s *g, const void *llr, bool llr_f64, int32_t batch,
                                int32_t max_iters, int32_t early_stop, uint8_t *hard, float *post, int32_t *iters,
                                void *ws, size_t ws_bytes, int32_t waves, hipStream_t stream,
                                const float *init_cv = nullptr, float *final_cv = nullptr);
// Stream form (stream.hip): readiness of a graph for it (device facts cached; an error
// if its word state exceeds LDS) and one enqueued decode using `counter` (device int).
ldpc_status stream_ready_for(ldpc_graph_s *g, int32_t threads);
ldpc_status launch_stream_decode(ldpc_graph_s *g, const void *llr, bool llr_f64, int32_t batch, int32_t max_iters,
                                 int32_t early_stop, uint8_t *hard_bits, float *posterior, int32_t *iters_used,
                                 int *counter, int32_t threads, hipStream_t stream);
size_t plain_workspace_bytes(const ldpc_graph_s *g, int32_t batch);  // full speed (decode.hip)
size_t plain_min_workspace_bytes(const ldpc_graph_s *g);             // one tile state at a time
// Split form (split.hip): workspace bytes and one enqueued decode (slices = 0: automatic).
size_t split_workspace_bytes(const ldpc_graph_s *g, int32_t batch);
ldpc_status launch_split_decode(const ldpc_graph_s *g, const void *llr, bool llr_f64, int32_t batch,
                                int32_t max_iters, int32_t early_stop, uint8_t *hard, float *post, int32_t *iters,
                                void *ws, int32_t slices, hipStream_t stream);
