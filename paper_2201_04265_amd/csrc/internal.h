// Internal declarations shared by the host-side sources of the decoder library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ldpc.h"

// Tanner graph: host arrays plus device copies.  Edge e (CSR order) joins
// check chk_of_edge[e] and variable col_idx[e]; var_edges lists, for each
// variable, its edge ids in ascending order (= ascending check index).
struct ldpc_graph_s {
  int32_t m = 0, n = 0;
  int64_t nnz = 0;
  int32_t dc_min = 0, dc_max = 0, dv_min = 0, dv_max = 0;
  std::vector<int32_t> row_ptr, col_idx, chk_of_edge, var_ptr, var_edges;
  int device = 0;
  int32_t *d_row_ptr = nullptr, *d_col_idx = nullptr, *d_var_ptr = nullptr, *d_var_edges = nullptr;
};

// Device view passed to kernels by value.
struct GraphDev {
  const int32_t *row_ptr;
  const int32_t *col_idx;
  const int32_t *var_ptr;
  const int32_t *var_edges;
  int32_t m, n, nnz;
  int32_t dc, dv;  // uniform degrees, or 0 when irregular
};

inline GraphDev graph_dev(const ldpc_graph_s *g) {
  GraphDev d;
  d.row_ptr = g->d_row_ptr;
  d.col_idx = g->d_col_idx;
  d.var_ptr = g->d_var_ptr;
  d.var_edges = g->d_var_edges;
  d.m = g->m;
  d.n = g->n;
  d.nnz = (int32_t)g->nnz;
  d.dc = g->dc_min == g->dc_max ? g->dc_max : 0;
  d.dv = g->dv_min == g->dv_max ? g->dv_max : 0;
  return d;
}

// Error reporting: thread-local detail of the last failure.
ldpc_status set_error(ldpc_status s, const std::string &msg);
ldpc_status hip_error(hipError_t e, const char *what);

#define LDPC_HIP_CHECK(call)                               \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return hip_error(e_, #call);     \
  } while (0)

constexpr int kTile = 64;  // codewords per tile: one per wavefront lane

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Plain decode launcher (decode.hip).
ldpc_status launch_plain_decode(const ldpc_graph_s *g, const void *llr, bool llr_f64, int32_t batch,
                                int32_t max_iters, int32_t early_stop, uint8_t *hard, float *post, int32_t *iters,
                                void *ws, size_t ws_bytes, int32_t waves, hipStream_t stream);
size_t plain_workspace_bytes(const ldpc_graph_s *g, int32_t batch);
