// Host-side graph construction and kernel layouts (see host_layout.h).
#include "host_layout.h"

#include <algorithm>
#include <climits>
#include <cstring>

namespace {
ldpc_status fail(std::string &err, ldpc_status s, const std::string &msg) {
  err = msg;
  return s;
}
}  // namespace

// Validate the compressed arrays and produce CSR with sorted rows.
static ldpc_status build_csr(int32_t m, int32_t n, ldpc_format fmt, const int32_t *ptr, const int32_t *idx, int64_t nnz,
                      std::vector<int32_t> &row_ptr, std::vector<int32_t> &col_idx, std::string &err) {
  const int32_t outer = fmt == LDPC_CSR ? m : n;
  const int32_t inner = fmt == LDPC_CSR ? n : m;
  if (ptr[0] != 0) return fail(err, LDPC_ERR_BAD_MATRIX, "ptr[0] must be 0");
  for (int32_t i = 0; i < outer; i++)
    if (ptr[i + 1] < ptr[i]) return fail(err, LDPC_ERR_BAD_MATRIX, "ptr is not non-decreasing");
  if ((int64_t)ptr[outer] != nnz) return fail(err, LDPC_ERR_BAD_MATRIX, "ptr[last] != nnz");
  for (int64_t k = 0; k < nnz; k++)
    if (idx[k] < 0 || idx[k] >= inner) return fail(err, LDPC_ERR_BAD_MATRIX, "index out of range");
  // counting sort into CSR; rows sorted by variable
  std::vector<int64_t> cnt((size_t)m + 1, 0);
  if (fmt == LDPC_CSR) {
    for (int32_t c = 0; c < m; c++) cnt[c + 1] = ptr[c + 1] - ptr[c];
  } else {
    for (int64_t k = 0; k < nnz; k++) cnt[idx[k] + 1]++;
  }
  for (int32_t c = 0; c < m; c++) cnt[c + 1] += cnt[c];
  row_ptr.assign((size_t)m + 1, 0);
  for (int32_t c = 0; c <= m; c++) row_ptr[c] = (int32_t)cnt[c];
  col_idx.assign((size_t)nnz, 0);
  if (fmt == LDPC_CSR) {
    std::memcpy(col_idx.data(), idx, (size_t)nnz * sizeof(int32_t));
  } else {
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int32_t v = 0; v < n; v++)
      for (int32_t k = ptr[v]; k < ptr[v + 1]; k++) col_idx[fill[idx[k]]++] = v;
  }
  for (int32_t c = 0; c < m; c++) {
    auto b = col_idx.begin() + row_ptr[c], e = col_idx.begin() + row_ptr[c + 1];
    std::sort(b, e);
    if (std::adjacent_find(b, e) != e) return fail(err, LDPC_ERR_BAD_MATRIX, "repeated entry in H");
  }
  return LDPC_OK;
}


ldpc_status graph_build_host(int32_t m, int32_t n, ldpc_format fmt, const int32_t *ptr, const int32_t *idx,
                             int64_t nnz, GraphHost &g, std::string &err) {
  if (m <= 0 || n <= 0) return fail(err, LDPC_ERR_BAD_MATRIX, "m and n must be positive");
  if (nnz < 0 || nnz > INT32_MAX) return fail(err, LDPC_ERR_BAD_MATRIX, "nnz out of range");
  g.m = m;
  g.n = n;
  g.nnz = nnz;
  ldpc_status st = build_csr(m, n, fmt, ptr, idx, nnz, g.row_ptr, g.col_idx, err);
  if (st != LDPC_OK) return st;
  g.dc_min = INT32_MAX;
  g.dc_max = 0;
  g.chk_of_edge.resize((size_t)nnz);
  for (int32_t c = 0; c < m; c++) {
    int32_t d = g.row_ptr[c + 1] - g.row_ptr[c];
    g.dc_min = std::min(g.dc_min, d);
    g.dc_max = std::max(g.dc_max, d);
    for (int32_t e = g.row_ptr[c]; e < g.row_ptr[c + 1]; e++) g.chk_of_edge[e] = c;
  }
  if (g.dc_min < 2) return fail(err, LDPC_ERR_BAD_MATRIX, "every check needs degree >= 2");
  g.var_ptr.assign((size_t)n + 1, 0);
  for (int64_t e = 0; e < nnz; e++) g.var_ptr[g.col_idx[e] + 1]++;
  g.dv_min = INT32_MAX;
  g.dv_max = 0;
  for (int32_t v = 0; v < n; v++) {
    g.dv_min = std::min(g.dv_min, g.var_ptr[v + 1]);
    g.dv_max = std::max(g.dv_max, g.var_ptr[v + 1]);
    g.var_ptr[v + 1] += g.var_ptr[v];
  }
  g.var_edges.assign((size_t)nnz, 0);
  {
    std::vector<int32_t> fill(g.var_ptr.begin(), g.var_ptr.end() - 1);
    for (int64_t e = 0; e < nnz; e++) g.var_edges[fill[g.col_idx[e]]++] = (int32_t)e;
  }
  if (g.dc_max > LDPC_MAX_CHECK_DEGREE || g.dv_max > LDPC_MAX_VAR_DEGREE)
    return fail(err, LDPC_ERR_UNSUPPORTED,
                "check degree > " + std::to_string(LDPC_MAX_CHECK_DEGREE) + " or variable degree > " +
                    std::to_string(LDPC_MAX_VAR_DEGREE));
  if ((int64_t)n * kTile > INT32_MAX || nnz * kTile > INT32_MAX)
    return fail(err, LDPC_ERR_UNSUPPORTED, "graph too large for 32-bit per-tile offsets");
  return LDPC_OK;
}

// Runtime check degrees: the checks, sorted by degree (ties in index order), are dealt
// in groups of 64, one group per wavefront pass of the check phase.  Group i starts at
// float start_i and holds entry j of its l-th check at start_i + 64 j + l, so the 64
// lanes of a wavefront read and write 64 consecutive floats (64 distinct LDS banks).
// A group spans 64 x its largest degree floats (the last one only up to its last
// entry); when every group has one degree (quasi-cyclic codes with a circulant size
// that is a multiple of 64, and every fixed degree) that is exactly the edge count.
// Each check reads and writes only its own entries, so the placement does not change
// any result.  For quasi-cyclic codes the stable sort keeps each block row's checks
// consecutive and 64-aligned, so the 64 variables a wavefront updates (consecutive
// columns of one circulant) also reach 64 distinct banks.
// The wavefronts of the kernel take these groups, and the groups of 64 consecutive
// variables, from a shared counter, so the tables list both costliest first (largest
// degree; ties in index order): taken in that order by whichever wavefront is free,
// the work of a phase spreads over the wavefronts as in longest-first list scheduling,
// whatever the workgroup size.  Which wavefront updates a check or a variable changes
// no result either.
StreamGroupLayout stream_group_layout(const GraphHost *g) {
  StreamGroupLayout L;
  const int m = g->m;
  std::vector<int32_t> order(m);
  for (int c = 0; c < m; ++c) order[c] = c;
  auto deg = [&](int c) { return g->row_ptr[c + 1] - g->row_ptr[c]; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return deg(a) < deg(b); });
  const int groups = (m + 63) / 64;
  L.slot.assign((size_t)groups * 64, 0);
  L.pos.assign((size_t)g->nnz, 0);
  int64_t start = 0;
  for (int gi = 0; gi < groups; ++gi) {
    const int cnt = std::min(64, m - 64 * gi);
    int dmax = 0;
    for (int l = 0; l < cnt; ++l) {
      const int c = order[64 * gi + l], d = deg(c);
      dmax = std::max(dmax, d);
      const int64_t base = start + l;
      L.slot[(size_t)64 * gi + l] = base < 65536 ? (int32_t)(base | ((int64_t)d << 16)) : 0;
      for (int j = 0; j < d; ++j) L.pos[(size_t)g->row_ptr[c] + j] = (int32_t)std::min<int64_t>(base + 64 * j, INT32_MAX);
    }
    start += gi + 1 < groups ? 64 * (int64_t)dmax : 64 * (int64_t)(dmax - 1) + cnt;
  }
  L.floats = start;
  // costliest first: the groups of checks (formed in ascending degree) and of variables
  auto costliest_first = [](const std::vector<int32_t> &deg) {
    std::vector<int32_t> order(deg.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int32_t)i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return deg[a] > deg[b]; });
    return order;
  };
  std::vector<int32_t> cdeg(groups, 0);
  for (size_t s = 0; s < L.slot.size(); ++s) cdeg[s / 64] = std::max(cdeg[s / 64], L.slot[s] >> 16);
  const std::vector<int32_t> corder = costliest_first(cdeg);
  std::vector<int32_t> formed = L.slot;
  for (int gi = 0; gi < groups; ++gi)
    std::copy(formed.begin() + 64 * (size_t)corder[gi], formed.begin() + 64 * (size_t)(corder[gi] + 1),
              L.slot.begin() + 64 * (size_t)gi);
  std::vector<int32_t> vdeg((g->n + 63) / 64, 0);
  for (int v = 0; v < g->n; ++v) vdeg[v >> 6] = std::max(vdeg[v >> 6], g->var_ptr[v + 1] - g->var_ptr[v]);
  L.var_order = costliest_first(vdeg);
  return L;
}

std::vector<int32_t> stream_group_table(const GraphHost *g, const StreamGroupLayout &L,
                                        const std::vector<int32_t> &var_off) {
  std::vector<int32_t> tab(L.slot);
  const size_t vgroups = L.var_order.size();
  tab.resize(tab.size() + 3 * vgroups);
  for (size_t i = 0; i < vgroups; ++i) {
    const int k = L.var_order[i], v0 = 64 * k, v1 = std::min(g->n, v0 + 64);
    int gd = 0, gmin = INT32_MAX;
    for (int v = v0; v < v1; ++v) {
      gd = std::max(gd, g->var_ptr[v + 1] - g->var_ptr[v]);
      gmin = std::min(gmin, g->var_ptr[v + 1] - g->var_ptr[v]);
    }
    const size_t start = tab.size();
    tab[L.slot.size() + 3 * i] = k;
    tab[L.slot.size() + 3 * i + 1] = (int32_t)start;
    tab[L.slot.size() + 3 * i + 2] = gmin == gd ? gd : -1;
    tab.resize(start + 64 * (size_t)(1 + (gd + 1) / 2), 0);
    for (int v = v0; v < v1; ++v) {
      tab[start + (v & 63)] = g->var_ptr[v + 1] - g->var_ptr[v];
      for (int32_t p = g->var_ptr[v]; p < g->var_ptr[v + 1]; ++p) {
        const int j = p - g->var_ptr[v];
        const uint32_t idx = (uint32_t)var_off[(size_t)p] / 4u;  // LDS float index, < 2^16
        uint32_t &w = reinterpret_cast<uint32_t &>(tab[start + 64 * (size_t)(1 + j / 2) + (v & 63)]);
        w |= (idx & 0xffffu) << (16 * (j & 1));
      }
    }
  }
  return tab;
}

// Where the check rows sit in LDS.  For a fixed check degree any order of the rows
// gives the same results (each check reads and writes only its own row), so the rows
// are placed in the order that keeps the LDS banks of the 64 variables a wavefront
// updates together as distinct as possible: swaps of two rows' places are kept when
// they do not raise the summed worst-bank load of the affected (64-variable block,
// edge rank) groups, ties going by the summed squared loads (a seeded local search,
// 100 swaps per check).  Returns each
// variable edge's LDS byte offset in var_edges order.
std::vector<int32_t> stream_edge_offsets(const GraphHost *g) {
  const size_t E = (size_t)g->nnz;
  std::vector<int32_t> off(E);
  if (g->m < 2) {
    for (size_t p = 0; p < E; ++p) off[p] = g->var_edges[p] * 4;
    return off;
  }
  constexpr int kBanks = 64;
  const int DC = g->dc_max, m = g->m, n = g->n, DV = std::max(1, g->dv_max);
  // group of edge e: (variable block of 64, rank of e among its variable's edges)
  std::vector<int32_t> grp(E);
  for (int v = 0; v < n; ++v)
    for (int32_t p = g->var_ptr[v]; p < g->var_ptr[v + 1]; ++p) grp[g->var_edges[p]] = (v >> 6) * DV + (p - g->var_ptr[v]);
  const size_t ngroups = (size_t)((n + 63) >> 6) * DV;
  std::vector<uint16_t> cnt(ngroups * kBanks, 0);
  std::vector<int32_t> slot(m);
  for (int c = 0; c < m; ++c) slot[c] = c;
  auto add = [&](int c, int s, int d) {
    for (int j = 0; j < DC; ++j) cnt[(size_t)grp[(size_t)c * DC + j] * kBanks + (s * DC + j) % kBanks] += d;
  };
  for (int c = 0; c < m; ++c) add(c, c, 1);
  // cost of a group: its worst bank load first, then the sum of squared loads (which
  // tells apart placements with the same worst load, so the search does not stall on
  // plateaus: 2.5 -> 2.1 average worst load for (3,6) n=4096 at the same swap count)
  auto cost = [&](int32_t gid) {
    const uint16_t *r = &cnt[(size_t)gid * kBanks];
    int w = 0;
    long q = 0;
    for (int b = 0; b < kBanks; ++b) {
      w = std::max<int>(w, r[b]);
      q += (long)r[b] * r[b];
    }
    return (long)w * 1000000L + q;
  };
  std::vector<int32_t> gs;
  gs.reserve(2 * DC);
  uint64_t x = 0x9E3779B97F4A7C15ull;  // xorshift64*, fixed seed: the same layout every time
  auto rnd = [&]() {
    x ^= x >> 12;
    x ^= x << 25;
    x ^= x >> 27;
    return (x * 0x2545F4914F6CDD1Dull) >> 33;
  };
  const long swaps = 100L * m;
  for (long it = 0; it < swaps; ++it) {
    const int a = (int)(rnd() % (uint64_t)m), b = (int)(rnd() % (uint64_t)m);
    if (a == b) continue;
    gs.clear();
    for (int j = 0; j < DC; ++j)
      for (int c : {a, b}) {
        const int32_t gid = grp[(size_t)c * DC + j];
        if (std::find(gs.begin(), gs.end(), gid) == gs.end()) gs.push_back(gid);
      }
    long before = 0, after = 0;
    for (int32_t gid : gs) before += cost(gid);
    add(a, slot[a], -1);
    add(b, slot[b], -1);
    add(a, slot[b], 1);
    add(b, slot[a], 1);
    for (int32_t gid : gs) after += cost(gid);
    if (after <= before) {
      std::swap(slot[a], slot[b]);
    } else {
      add(a, slot[b], -1);
      add(b, slot[a], -1);
      add(a, slot[a], 1);
      add(b, slot[b], 1);
    }
  }
  for (size_t p = 0; p < E; ++p) {
    const int32_t e = g->var_edges[p];
    off[p] = (slot[e / DC] * DC + e % DC) * 4;
  }
  return off;
}

int64_t stream_x_floats(const GraphHost *g) {
  if (kernel_kind(g) < KIND_G8) return g->nnz;  // fixed degrees: one row per check
  // the group spans of stream_group_layout, from the sorted degrees alone
  std::vector<int32_t> deg(g->m);
  for (int c = 0; c < g->m; ++c) deg[c] = g->row_ptr[c + 1] - g->row_ptr[c];
  std::sort(deg.begin(), deg.end());
  int64_t floats = 0;
  for (int i0 = 0; i0 < g->m; i0 += 64) {
    const int cnt = std::min(64, g->m - i0), dmax = deg[i0 + cnt - 1];
    floats += i0 + 64 < g->m ? 64 * (int64_t)dmax : 64 * (int64_t)(dmax - 1) + cnt;
  }
  return floats;
}

// Reduced row echelon form of H over GF(2), pivots from the last column down.
void systematic_form(const GraphHost *g, std::vector<int32_t> &pivots, std::vector<uint64_t> &rows, int &W) {
  const int m = g->m, n = g->n;
  W = (n + 63) / 64;
  rows.assign((size_t)m * W, 0);
  for (int c = 0; c < m; ++c)
    for (int32_t p = g->row_ptr[c]; p < g->row_ptr[c + 1]; ++p) {
      const int v = g->col_idx[p];
      rows[(size_t)c * W + (v >> 6)] |= 1ull << (v & 63);
    }
  int rank = 0;
  pivots.clear();
  for (int col = n - 1; col >= 0 && rank < m; --col) {
    const int cw = col >> 6;
    const uint64_t cb = 1ull << (col & 63);
    int p = -1;
    for (int r = rank; r < m; ++r)
      if (rows[(size_t)r * W + cw] & cb) {
        p = r;
        break;
      }
    if (p < 0) continue;
    if (p != rank)
      std::swap_ranges(rows.begin() + (size_t)p * W, rows.begin() + (size_t)(p + 1) * W,
                       rows.begin() + (size_t)rank * W);
    // the pivot row is zero right of col (earlier pivots eliminated, skipped columns
    // are zero in every remaining row), so only words 0..cw change
    const uint64_t *pr = &rows[(size_t)rank * W];
    for (int r = 0; r < m; ++r) {
      if (r == rank) continue;
      uint64_t *rr = &rows[(size_t)r * W];
      if (rr[cw] & cb)
        for (int x = 0; x <= cw; ++x) rr[x] ^= pr[x];
    }
    pivots.push_back(col);
    ++rank;
  }
}

