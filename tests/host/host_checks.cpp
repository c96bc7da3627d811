// Host-side checks of the graph builder and the kernel layouts (host_layout.cpp), built with
// the address and undefined-behaviour sanitizers by tests/test_host_sanitizers.py.  Every
// check is a property the layouts must have, on seeded random parity-check matrices.
#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "../../paper_2201_04265_amd/csrc/host_layout.h"

static int failures = 0;
#define CHECK(cond)                                                             \
  do {                                                                          \
    if (!(cond)) {                                                              \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond);   \
      ++failures;                                                               \
    }                                                                           \
  } while (0)

// Random H (m x n) as sorted CSR rows with check degrees in [dmin, dmax].
static void random_h(std::mt19937 &r, int m, int n, int dmin, int dmax, std::vector<int32_t> &ptr,
                     std::vector<int32_t> &idx) {
  ptr.assign(1, 0);
  idx.clear();
  std::vector<int> cols(n);
  for (int v = 0; v < n; ++v) cols[v] = v;
  for (int c = 0; c < m; ++c) {
    const int d = std::min(n, dmin + (int)(r() % (unsigned)(dmax - dmin + 1)));
    std::shuffle(cols.begin(), cols.end(), r);
    std::vector<int> row(cols.begin(), cols.begin() + d);
    std::sort(row.begin(), row.end());
    idx.insert(idx.end(), row.begin(), row.end());
    ptr.push_back((int32_t)idx.size());
  }
}

static void to_csc(int m, int n, const std::vector<int32_t> &ptr, const std::vector<int32_t> &idx,
                   std::vector<int32_t> &cptr, std::vector<int32_t> &cidx) {
  cptr.assign(n + 1, 0);
  for (int32_t v : idx) cptr[v + 1]++;
  for (int v = 0; v < n; ++v) cptr[v + 1] += cptr[v];
  cidx.assign(idx.size(), 0);
  std::vector<int32_t> fill(cptr.begin(), cptr.end() - 1);
  for (int c = 0; c < m; ++c)
    for (int32_t p = ptr[c]; p < ptr[c + 1]; ++p) cidx[fill[idx[p]]++] = c;
}

static void check_graph(const GraphHost &g, const std::vector<int32_t> &ptr, const std::vector<int32_t> &idx) {
  CHECK(g.row_ptr == ptr && g.col_idx == idx);
  CHECK((int64_t)g.chk_of_edge.size() == g.nnz && (int64_t)g.var_edges.size() == g.nnz);
  for (int c = 0; c < g.m; ++c)
    for (int32_t e = g.row_ptr[c]; e < g.row_ptr[c + 1]; ++e) CHECK(g.chk_of_edge[e] == c);
  std::vector<int> seen(g.nnz, 0);
  for (int v = 0; v < g.n; ++v) {
    for (int32_t p = g.var_ptr[v]; p < g.var_ptr[v + 1]; ++p) {
      const int32_t e = g.var_edges[p];
      CHECK(e >= 0 && e < g.nnz);
      if (e < 0 || e >= g.nnz) continue;
      CHECK(g.col_idx[e] == v);
      ++seen[e];
      if (p > g.var_ptr[v]) CHECK(g.chk_of_edge[g.var_edges[p - 1]] < g.chk_of_edge[e]);
    }
  }
  for (int x : seen) CHECK(x == 1);
}

static void check_layouts(const GraphHost &g) {
  const int kind = kernel_kind(&g);
  if (kind >= KIND_G8) {
    const StreamGroupLayout L = stream_group_layout(&g);
    CHECK(L.floats == stream_x_floats(&g));
    CHECK((int64_t)L.pos.size() == g.nnz && L.slot.size() % 64 == 0);
    std::set<int32_t> used;
    for (int32_t p : L.pos) {
      CHECK(p >= 0 && p < L.floats);
      used.insert(p);
    }
    CHECK((int64_t)used.size() == g.nnz);
    // every check sits in one slot with its own degree; its entries step by 64
    std::vector<int> slot_of(g.m, -1);
    for (int c = 0; c < g.m; ++c) {
      const int32_t e0 = g.row_ptr[c], d = g.row_ptr[c + 1] - e0;
      for (int j = 1; j < d; ++j) CHECK(L.pos[e0 + j] == L.pos[e0] + 64 * j);
      int hits = 0;
      for (size_t s = 0; s < L.slot.size(); ++s)
        if (L.slot[s] && (L.slot[s] & 0xffff) == L.pos[e0] && (L.slot[s] >> 16) == d) ++hits;
      CHECK(hits == 1);
    }
    // the groups of 64 slots by non-increasing largest degree
    const size_t groups = L.slot.size() / 64;
    int prev = INT_MAX;
    for (size_t gi = 0; gi < groups; ++gi) {
      int d = 0;
      for (int l = 0; l < 64; ++l) d = std::max(d, L.slot[64 * gi + l] >> 16);
      CHECK(d <= prev);
      prev = d;
    }
    // the groups of 64 variables: a permutation, by non-increasing largest degree
    const int vgroups = (g.n + 63) / 64;
    CHECK((int)L.var_order.size() == vgroups);
    std::vector<int> taken(vgroups, 0);
    prev = INT_MAX;
    for (int32_t k : L.var_order) {
      CHECK(k >= 0 && k < vgroups);
      if (k < 0 || k >= vgroups) continue;
      ++taken[k];
      int d = 0;
      for (int v = 64 * k; v < std::min(g.n, 64 * k + 64); ++v) d = std::max(d, g.var_ptr[v + 1] - g.var_ptr[v]);
      CHECK(d <= prev);
      prev = d;
    }
    for (int x : taken) CHECK(x == 1);
    // the kernel's table: the slots, the order entries, and the rows of every variable group
    std::vector<int32_t> off((size_t)g.nnz);
    for (size_t p = 0; p < off.size(); ++p) off[p] = L.pos[(size_t)g.var_edges[p]] * 4;
    const std::vector<int32_t> tab = stream_group_table(&g, L, off);
    const size_t S = L.slot.size();
    CHECK(tab.size() >= S + 3 * (size_t)vgroups);
    for (size_t s = 0; s < S; ++s) CHECK(tab[s] == L.slot[s]);
    size_t end = S + 3 * (size_t)vgroups;
    for (int i = 0; i < vgroups; ++i) {
      const int k = tab[S + 3 * i], start = tab[S + 3 * i + 1], ud = tab[S + 3 * i + 2];
      CHECK(k == L.var_order[i]);
      CHECK((size_t)start == end);  // rows follow each other in the order's sequence
      int gd = 0, gmin = INT_MAX;
      for (int v = 64 * k; v < std::min(g.n, 64 * k + 64); ++v) {
        const int d = g.var_ptr[v + 1] - g.var_ptr[v];
        gd = std::max(gd, d);
        gmin = std::min(gmin, d);
        CHECK(tab[(size_t)start + (v & 63)] == d);
        for (int j = 0; j < d; ++j) {
          const uint32_t w = (uint32_t)tab[(size_t)start + 64 * (1 + j / 2) + (v & 63)];
          CHECK(((w >> (16 * (j & 1))) & 0xffffu) * 4u == (uint32_t)off[(size_t)g.var_ptr[v] + j]);
        }
        if (d % 2 == 1)  // the unused half of the last entry stays 0
          CHECK(((uint32_t)tab[(size_t)start + 64 * (1 + d / 2) + (v & 63)] >> 16) == 0u);
      }
      CHECK(ud == (gmin == gd ? gd : -1));
      end = (size_t)start + 64 * (size_t)(1 + (gd + 1) / 2);
    }
    CHECK(tab.size() == end);
  } else {
    const std::vector<int32_t> off = stream_edge_offsets(&g);
    CHECK((int64_t)off.size() == g.nnz && stream_x_floats(&g) == g.nnz);
    std::set<int32_t> used;
    for (int32_t o : off) {
      CHECK(o % 4 == 0 && o >= 0 && o < 4 * g.nnz);
      used.insert(o);
    }
    CHECK((int64_t)used.size() == g.nnz);
    // the edges of one check fill one whole row of dc floats, in their order
    const int dc = g.dc_max;
    std::vector<int32_t> at(g.nnz);
    for (int64_t p = 0; p < g.nnz; ++p) at[g.var_edges[p]] = off[p] / 4;
    for (int c = 0; c < g.m; ++c) {
      CHECK(at[(size_t)c * dc] % dc == 0);
      for (int j = 1; j < dc; ++j) CHECK(at[(size_t)c * dc + j] == at[(size_t)c * dc] + j);
    }
  }
}

// Codewords from the reduced rows: message bits on the non-pivot columns, each pivot bit the
// parity of its row's message bits; every codeword must satisfy H c = 0 (Eq. 1).
static void check_systematic(const GraphHost &g, std::mt19937 &r) {
  std::vector<int32_t> piv;
  std::vector<uint64_t> rows;
  int W = 0;
  systematic_form(&g, piv, rows, W);
  const int rank = (int)piv.size();
  CHECK(rank <= g.m);
  std::vector<char> is_piv(g.n, 0);
  for (int32_t p : piv) {
    CHECK(p >= 0 && p < g.n);
    if (p >= 0 && p < g.n) is_piv[p] = 1;
  }
  for (int t = 0; t < 8; ++t) {
    std::vector<uint8_t> c(g.n, 0);
    for (int v = 0; v < g.n; ++v)
      if (!is_piv[v]) c[v] = r() & 1;
    for (int i = 0; i < rank; ++i) {
      int par = 0;
      for (int v = 0; v < g.n; ++v)
        if (!is_piv[v] && ((rows[(size_t)i * W + (v >> 6)] >> (v & 63)) & 1ull)) par ^= c[v];
      c[piv[i]] = (uint8_t)par;
    }
    for (int ch = 0; ch < g.m; ++ch) {
      int s = 0;
      for (int32_t p = g.row_ptr[ch]; p < g.row_ptr[ch + 1]; ++p) s ^= c[g.col_idx[p]];
      CHECK(s == 0);
    }
  }
}

static ldpc_status build(int m, int n, ldpc_format f, const std::vector<int32_t> &ptr, const std::vector<int32_t> &idx,
                         GraphHost &g) {
  std::string err;
  return graph_build_host(m, n, f, ptr.data(), idx.data(), (int64_t)idx.size(), g, err);
}

int main() {
  std::mt19937 r(2201);
  // valid matrices: fixed degree pairs (regular rows) and irregular ones, CSR and CSC
  struct Case {
    int m, n, dmin, dmax;
  };
  const Case cases[] = {{48, 96, 6, 6},   {64, 256, 4, 4},  {30, 120, 12, 12}, {40, 200, 15, 15},
                        {37, 101, 2, 20}, {80, 160, 3, 32}, {5, 7, 2, 3},      {130, 300, 5, 24}};
  for (const Case &k : cases) {
    std::vector<int32_t> ptr, idx, cptr, cidx;
    random_h(r, k.m, k.n, k.dmin, k.dmax, ptr, idx);
    GraphHost g, gc;
    const ldpc_status st = build(k.m, k.n, LDPC_CSR, ptr, idx, g);
    to_csc(k.m, k.n, ptr, idx, cptr, cidx);
    const ldpc_status stc = build(k.m, k.n, LDPC_CSC, cptr, cidx, gc);
    const bool unsupported = g.dv_max > LDPC_MAX_VAR_DEGREE;
    CHECK(st == (unsupported ? LDPC_ERR_UNSUPPORTED : LDPC_OK) && stc == st);
    if (st != LDPC_OK) continue;
    check_graph(g, ptr, idx);
    check_graph(gc, ptr, idx);
    check_layouts(g);
    check_systematic(g, r);
  }
  // malformed matrices are refused with the documented status
  {
    GraphHost g;
    std::vector<int32_t> ptr{0, 2, 4}, idx{0, 1, 1, 2};
    CHECK(build(2, 3, LDPC_CSR, ptr, idx, g) == LDPC_OK);
    std::vector<int32_t> bad_first{1, 2, 4};
    CHECK(build(2, 3, LDPC_CSR, bad_first, idx, g) == LDPC_ERR_BAD_MATRIX);
    std::vector<int32_t> dec{0, 3, 2};
    CHECK(build(2, 3, LDPC_CSR, dec, std::vector<int32_t>{0, 1, 2}, g) == LDPC_ERR_BAD_MATRIX);
    std::vector<int32_t> oor{0, 1, 5, 1};
    CHECK(build(2, 3, LDPC_CSR, ptr, oor, g) == LDPC_ERR_BAD_MATRIX);
    std::vector<int32_t> dup{0, 0, 1, 2};
    CHECK(build(2, 3, LDPC_CSR, ptr, dup, g) == LDPC_ERR_BAD_MATRIX);
    std::vector<int32_t> p1{0, 1, 3}, i1{0, 1, 2};
    CHECK(build(2, 3, LDPC_CSR, p1, i1, g) == LDPC_ERR_BAD_MATRIX);  // a check of degree 1
    std::vector<int32_t> pw{0, 33}, iw(33);
    for (int v = 0; v < 33; ++v) iw[v] = v;
    CHECK(build(1, 40, LDPC_CSR, pw, iw, g) == LDPC_ERR_UNSUPPORTED);  // check degree 33
    CHECK(build(0, 3, LDPC_CSR, std::vector<int32_t>{0}, std::vector<int32_t>{}, g) == LDPC_ERR_BAD_MATRIX);
  }
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("host checks ok\n");
  return 0;
}
