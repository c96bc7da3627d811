// Host-side construction of the Tanner graph and of the layouts the kernels use:
// plain C++ with no device code, so that it also builds on its own with the host
// address and undefined-behaviour sanitizers (the CPU tests do that).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ldpc.h"

constexpr int kTile = 64;  // codewords per tile: one per wavefront lane

// Tanner graph of H (Sec. II-B, Fig. 1) as host arrays.  Edge e (CSR order) joins check
// chk_of_edge[e] and variable col_idx[e]; var_edges lists, for each variable, its edge
// ids in ascending order (= ascending check index).
struct GraphHost {
  int32_t m = 0, n = 0;
  int64_t nnz = 0;
  int32_t dc_min = 0, dc_max = 0, dv_min = 0, dv_max = 0;
  std::vector<int32_t> row_ptr, col_idx, chk_of_edge, var_ptr, var_edges;
};

// Validates the compressed arrays (fmt: CSR over checks or CSC over variables), builds the
// graph and checks the kernels' limits.  On failure returns the status and sets err.
ldpc_status graph_build_host(int32_t m, int32_t n, ldpc_format fmt, const int32_t *ptr, const int32_t *idx,
                             int64_t nnz, GraphHost &g, std::string &err);

// Degree specialisations compiled for the kernels: fixed (dc, dv) pairs, then
// generic kernels for irregular codes up to a maximum check degree.  The degree-24
// class also bounds the variable degree (12: quasi-cyclic protographs stay below it), so
// that its register arrays leave room for the stream form's prefetch of the next
// variables; codes with a variable of degree 13 to 16 take the degree-32 class.
constexpr int kG24MaxVarDegree = 12;
enum KernelKind : int32_t {
  KIND_6_3 = 0,
  KIND_4_3,
  KIND_12_3,
  KIND_15_3,
  KIND_12_6,
  KIND_12_9,
  KIND_G8,
  KIND_G16,
  KIND_G24,
  KIND_G32,
  KIND_COUNT
};

inline int32_t kernel_kind(const GraphHost *g) {
  const bool reg = g->dc_min == g->dc_max && g->dv_min == g->dv_max;
  if (reg) {
    const int dc = g->dc_max, dv = g->dv_max;
    if (dc == 6 && dv == 3) return KIND_6_3;
    if (dc == 4 && dv == 3) return KIND_4_3;
    if (dc == 12 && dv == 3) return KIND_12_3;
    if (dc == 15 && dv == 3) return KIND_15_3;
    if (dc == 12 && dv == 6) return KIND_12_6;
    if (dc == 12 && dv == 9) return KIND_12_9;
  }
  if (g->dc_max <= 8) return KIND_G8;
  if (g->dc_max <= 16) return KIND_G16;
  if (g->dc_max <= 24 && g->dv_max <= kG24MaxVarDegree) return KIND_G24;
  return KIND_G32;
}


// Stream form, runtime check degrees: LDS placement of the checks' rows, 64 at a time.
struct StreamGroupLayout {
  std::vector<int32_t> slot;       // [64 x groups]: start float | degree << 16 (0 = no check),
                                   // groups listed by descending degree
  std::vector<int32_t> pos;        // [nnz]: float index of each edge (CSR order)
  std::vector<int32_t> var_order;  // [ceil(n / 64)]: groups of 64 variables, costliest first
  int64_t floats = 0;
};
StreamGroupLayout stream_group_layout(const GraphHost *g);
// Stream form, runtime degrees: the kernel's table.  The check slots of L; then, per position
// of L.var_order, the group, where its rows start and its degree when all its variables share
// one (else -1); then the rows, group by group: the 64 lanes' degrees, then their edges' LDS
// float indices (var_off / 4, var_off in var_edges order), two to an entry: index j of lane l
// in bits 16 (j mod 2) .. +15 of entry start + 64 (1 + j / 2) + l, so that a wavefront reads
// each row as one contiguous 256-byte segment (64 x (1 + half the group's largest degree,
// rounded up) entries).  LDS indices fit 16 bits: a workgroup's LDS holds fewer floats.
std::vector<int32_t> stream_group_table(const GraphHost *g, const StreamGroupLayout &L,
                                        const std::vector<int32_t> &var_off);
// Stream form, fixed check degrees: each variable edge's LDS byte offset (var_edges order)
// after the bank-spreading placement of the rows.
std::vector<int32_t> stream_edge_offsets(const GraphHost *g);
// Floats of the stream form's per-word message array for this graph's layout.
int64_t stream_x_floats(const GraphHost *g);

// Reduced row echelon form of H over GF(2), pivot columns taken from the last column down;
// rows holds the m reduced rows bit-packed (W 64-bit words each).
void systematic_form(const GraphHost *g, std::vector<int32_t> &pivots, std::vector<uint64_t> &rows, int &W);
