// Tanner-graph layout builder and the C-ABI shell (status strings, errors).
//
// The graph of Sec. II-B (Fig. 1): one edge per 1 in H.  Input is CSR or CSC
// host arrays; the builder validates them, numbers the edges check-major
// (CSR order), derives each variable's edge list and uploads all index
// arrays to the current device once.
#include <algorithm>
#include <cstring>
#include <new>

#include "internal.h"

namespace {
thread_local std::string g_last_error;
}

ldpc_status set_error(ldpc_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

ldpc_status hip_error(hipError_t e, const char *what) {
  return set_error(LDPC_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

extern "C" const char *ldpc_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *ldpc_status_string(ldpc_status s) {
  switch (s) {
    case LDPC_OK: return "ok";
    case LDPC_ERR_INVALID_ARG: return "invalid argument";
    case LDPC_ERR_BAD_MATRIX: return "bad parity-check matrix";
    case LDPC_ERR_OUT_OF_MEMORY: return "out of memory";
    case LDPC_ERR_DEVICE: return "device error";
    case LDPC_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

namespace {

void free_device(ldpc_graph_s *g) {
  if (g->d_row_ptr) (void)hipFree(g->d_row_ptr);
  if (g->d_col_idx) (void)hipFree(g->d_col_idx);
  if (g->d_var_ptr) (void)hipFree(g->d_var_ptr);
  if (g->d_var_edges) (void)hipFree(g->d_var_edges);
  if (g->d_var_xoff) (void)hipFree(g->d_var_xoff);
  if (g->d_xslot) (void)hipFree(g->d_xslot);
  g->d_row_ptr = g->d_col_idx = g->d_var_ptr = g->d_var_edges = g->d_var_xoff = g->d_xslot = nullptr;
}

std::vector<int32_t> byte_offsets(const std::vector<int32_t> &edges) {
  std::vector<int32_t> o(edges.size());
  for (size_t i = 0; i < edges.size(); ++i) o[i] = edges[i] * 4;
  return o;
}

ldpc_status upload(const std::vector<int32_t> &h, int32_t **d) {
  size_t bytes = std::max<size_t>(h.size(), 1) * sizeof(int32_t);
  hipError_t e = hipMalloc((void **)d, bytes);
  if (e != hipSuccess) {
    *d = nullptr;
    return set_error(LDPC_ERR_OUT_OF_MEMORY, std::string("hipMalloc graph: ") + hipGetErrorString(e));
  }
  if (!h.empty()) LDPC_HIP_CHECK(hipMemcpy(*d, h.data(), h.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  return LDPC_OK;
}

}  // namespace

extern "C" ldpc_status ldpc_graph_create(int32_t m, int32_t n, ldpc_format fmt, const int32_t *ptr,
                                         const int32_t *idx, int64_t nnz, ldpc_graph_t *out) {
  if (!out) return set_error(LDPC_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (fmt != LDPC_CSR && fmt != LDPC_CSC) return set_error(LDPC_ERR_INVALID_ARG, "unknown format");
  if (m <= 0 || n <= 0) return set_error(LDPC_ERR_BAD_MATRIX, "m and n must be positive");
  if (nnz < 0 || nnz > INT32_MAX) return set_error(LDPC_ERR_BAD_MATRIX, "nnz out of range");
  ldpc_graph_s *g = new (std::nothrow) ldpc_graph_s();
  if (!g) return set_error(LDPC_ERR_OUT_OF_MEMORY, "graph allocation");
  if (!ptr || (nnz > 0 && !idx)) {
    delete g;
    return set_error(LDPC_ERR_INVALID_ARG, "ptr/idx is NULL");
  }
  std::string err;
  ldpc_status st = graph_build_host(m, n, fmt, ptr, idx, nnz, *g, err);
  if (st != LDPC_OK) {
    delete g;
    return set_error(st, err);
  }
  g->stream_x_floats = stream_x_floats(g);
  hipError_t e = hipGetDevice(&g->device);
  if (e != hipSuccess) {
    delete g;
    return hip_error(e, "hipGetDevice");
  }
  if ((st = upload(g->row_ptr, &g->d_row_ptr)) != LDPC_OK || (st = upload(g->col_idx, &g->d_col_idx)) != LDPC_OK ||
      (st = upload(g->var_ptr, &g->d_var_ptr)) != LDPC_OK || (st = upload(g->var_edges, &g->d_var_edges)) != LDPC_OK ||
      (st = upload(byte_offsets(g->var_edges), &g->d_var_xoff)) != LDPC_OK) {
    free_device(g);
    delete g;
    return st;
  }
  *out = g;
  return LDPC_OK;
}

extern "C" ldpc_status ldpc_graph_destroy(ldpc_graph_t g) {
  if (!g) return set_error(LDPC_ERR_INVALID_ARG, "graph is NULL");
  free_device(g);
  delete g;
  return LDPC_OK;
}

extern "C" ldpc_status ldpc_graph_info(ldpc_graph_t g, int32_t *m, int32_t *n, int64_t *edges, int32_t *max_check_deg,
                                       int32_t *max_var_deg) {
  if (!g) return set_error(LDPC_ERR_INVALID_ARG, "graph is NULL");
  if (m) *m = g->m;
  if (n) *n = g->n;
  if (edges) *edges = g->nnz;
  if (max_check_deg) *max_check_deg = g->dc_max;
  if (max_var_deg) *max_var_deg = g->dv_max;
  return LDPC_OK;
}

extern "C" ldpc_status ldpc_graph_edges(ldpc_graph_t g, int32_t *check_of_edge, int32_t *var_of_edge) {
  if (!g) return set_error(LDPC_ERR_INVALID_ARG, "graph is NULL");
  if (check_of_edge && g->nnz) std::memcpy(check_of_edge, g->chk_of_edge.data(), g->nnz * sizeof(int32_t));
  if (var_of_edge && g->nnz) std::memcpy(var_of_edge, g->col_idx.data(), g->nnz * sizeof(int32_t));
  return LDPC_OK;
}

extern "C" ldpc_status ldpc_decode_workspace_size(ldpc_graph_t g, int32_t batch, uint32_t flags, size_t *bytes) {
  if (!g || !bytes) return set_error(LDPC_ERR_INVALID_ARG, "graph or bytes is NULL");
  if (batch < 0) return set_error(LDPC_ERR_INVALID_ARG, "batch < 0");
  if (flags & ~LDPC_LLR_F64) return set_error(LDPC_ERR_INVALID_ARG, "unknown flag");
  *bytes = plain_workspace_bytes(g, batch);
  return LDPC_OK;
}

static ldpc_status decode_common(ldpc_graph_t g, const void *llr, int32_t batch, int32_t max_iters,
                                 int32_t early_stop, uint32_t flags, uint8_t *hard, float *post, int32_t *iters,
                                 void *ws, size_t ws_bytes, int32_t waves, hipStream_t stream,
                                 const float *init_cv = nullptr, float *final_cv = nullptr) {
  if (!g) return set_error(LDPC_ERR_INVALID_ARG, "graph is NULL");
  if (batch < 0) return set_error(LDPC_ERR_INVALID_ARG, "batch < 0");
  if (max_iters < 0) return set_error(LDPC_ERR_INVALID_ARG, "max_iters < 0");
  if (flags & ~LDPC_LLR_F64) return set_error(LDPC_ERR_INVALID_ARG, "unknown flag");
  if (waves < 1 || waves > 16) return set_error(LDPC_ERR_INVALID_ARG, "waves must be in 1..16");
  if (batch == 0) return LDPC_OK;
  if (!llr || !hard || !post || !iters || !ws) return set_error(LDPC_ERR_INVALID_ARG, "NULL buffer");
  if (((uintptr_t)ws & 255) != 0) return set_error(LDPC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < plain_min_workspace_bytes(g))
    return set_error(LDPC_ERR_INVALID_ARG, "workspace too small for one 64-word tile state");
  return launch_plain_decode(g, llr, (flags & LDPC_LLR_F64) != 0, batch, max_iters, early_stop, hard, post, iters,
                             ws, ws_bytes, waves, stream, init_cv, final_cv);
}

extern "C" ldpc_status ldpc_decode(ldpc_graph_t g, const void *llr, int32_t batch, int32_t max_iters,
                                   int32_t early_stop, uint32_t flags, uint8_t *hard_bits, float *posterior,
                                   int32_t *iters_used, void *workspace, size_t ws_bytes, hipStream_t stream) {
  // 16 waves per tile: more loads in flight per compute unit (against 8 waves: 1.5x on the
  // n=11264 quasi-cyclic code, 1.4x on n=1032 Table I batches, 1.06x on (3,6) n=4096)
  return decode_common(g, llr, batch, max_iters, early_stop, flags, hard_bits, posterior, iters_used, workspace,
                       ws_bytes, 16, stream);
}

extern "C" ldpc_status ldpc_decode_config(ldpc_graph_t g, const void *llr, int32_t batch, int32_t max_iters,
                                          int32_t early_stop, uint32_t flags, uint8_t *hard_bits, float *posterior,
                                          int32_t *iters_used, void *workspace, size_t ws_bytes, int32_t waves,
                                          hipStream_t stream) {
  return decode_common(g, llr, batch, max_iters, early_stop, flags, hard_bits, posterior, iters_used, workspace,
                       ws_bytes, waves, stream);
}

extern "C" ldpc_status ldpc_decode_ex(ldpc_graph_t g, const void *llr, int32_t batch, int32_t max_iters,
                                      int32_t early_stop, uint32_t flags, const float *init_cv, float *final_cv,
                                      uint8_t *hard_bits, float *posterior, int32_t *iters_used, void *workspace,
                                      size_t ws_bytes, hipStream_t stream) {
  if (g && g->nnz == 0 && (init_cv || final_cv))
    return set_error(LDPC_ERR_INVALID_ARG, "a graph without edges has no c->v state");
  return decode_common(g, llr, batch, max_iters, early_stop, flags, hard_bits, posterior, iters_used, workspace,
                       ws_bytes, 16, stream, init_cv, final_cv);
}
