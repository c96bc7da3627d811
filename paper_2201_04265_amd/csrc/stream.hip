// Stream form: one word per workgroup, the decoding state in LDS.
//
// Sec. III-B spreads one word's Tanner graph over many workers ("stream
// processing") and finds the exchange of messages between workers, every
// half-iteration, to be its cost.  Inside one compute unit that exchange is an
// LDS barrier, so here a workgroup owns one word at a time: its threads take
// the checks (check phase) and then the variables (variable phase), in the
// interleaved order of Algorithm 1 (check c and variable v on thread c mod NT and
// v mod NT; for runtime degrees the wavefronts take groups of 64 checks or variables,
// costliest first, from a counter per phase), and every message stays in LDS.
// Workgroups are persistent and take the next word from an atomic counter when
// theirs stops, so a word that needs few iterations never waits for another.
//
// LDS per word:
//   X [nnz] FP32  one message per edge, updated in place: the check phase reads the
//                 v->c message (Eq. 6, clamped; stored with its variable's decision) and
//                 leaves the c->v message (Eq. 5); the variable phase reads that and
//                 leaves the next v->c message.  Each edge is touched by its own
//                 check, then by its own variable.  Fixed check degrees keep each
//                 check's messages as one row (rows placed for distinct LDS banks in
//                 the variable phase); runtime degrees interleave the rows of the 64
//                 checks one wavefront updates together (see stream_group_layout).
// The channel LLRs are re-read from the caller's buffer in every variable phase and the
// posterior of each variable phase (Eq. 7) goes straight to the caller's output row
// (both coalesced, and the rewrites of a row stay in L2), so a word needs 4 bytes of
// LDS per edge: 48 KB for (3,6) n=4096, three words per compute unit, and codes up to
// about 40 000 edges fit.
// The check phase tests the syndrome of the decisions its messages carry (Eq. 1)
// while it computes new messages.  Per edge the arithmetic and its order are those
// of the plain decoder, so the outputs are identical to it bit for bit.
#include "internal.h"
#include "tile.h"

namespace ldpc {

// X at LDS address 0 (so an edge's byte offset is its LDS address), then the word
// index, the two work counters of the runtime-degree phases and the per-wave syndrome
// flags.
inline size_t stream_x_bytes(const ldpc_graph_s *g) { return ((size_t)g->stream_x_floats * 4 + 15) & ~size_t(15); }
inline size_t stream_lds_bytes(const ldpc_graph_s *g) { return stream_x_bytes(g) + 80; }

// Workgroup size limit per degree pair: every kernel fits the 128-VGPR budget of a
// 1024-thread workgroup (the runtime-degree kernels keep half of their prefix pairs in
// the check's LDS row, see check_core_row).
template <int DC>
constexpr int kStreamMaxThreads = 1024;

template <int DC, int DV, bool F64>
__global__ void __launch_bounds__(kStreamMaxThreads<DC>)
    stream_decode_kernel(GraphDev g, const float *__restrict__ llr32, const double *__restrict__ llr64, int B,
                         int max_iters, int early_stop, int *counter, uint8_t *__restrict__ hard,
                         float *__restrict__ post, int32_t *__restrict__ iters, const int32_t *__restrict__ xslot,
                         int xslots, int xbytes) {
  constexpr int DCM = DC > 0 ? DC : -DC;
  constexpr int DVM = DV > 0 ? DV : -DV;
  extern __shared__ __align__(16) float smem[];
  float *X = smem;
  int *s_misc = (int *)((char *)smem + xbytes);
  int &s_word = s_misc[0];
  int *s_next = s_misc + 1;   // [2] runtime degrees: next group of the check / variable phase
  int *s_unsat = s_misc + 4;  // [16] per wavefront: some check of the word is unsatisfied
  const int t = threadIdx.x, NT = blockDim.x;
  const int wave = wave_id(), W = NT >> 6;
  const size_t n = (size_t)g.n;

  // Runtime degrees: a wavefront takes the next group of 64 checks (variables) from the
  // phase's counter; the tables list the groups costliest first (stream_group_layout).
  // Each counter is cleared by thread 0 in the other phase, between the barriers that
  // end its own phases, so no wavefront reads it meanwhile.
  auto next_group = [&](int *ctr) {
    int k = 0;
    if ((t & 63) == 0) k = atomicAdd(ctr, 1);
    return __builtin_amdgcn_readfirstlane(k);
  };

  for (;;) {
    if (t == 0) {
      s_word = atomicAdd(counter, 1);
      s_next[0] = 0;
      s_next[1] = 0;
    }
    lds_barrier();
    const int word = s_word;
    if (word >= B) break;  // same value in every thread
    const size_t base = (size_t)word * n;

    // ingest: posterior = channel LLRs, first messages X = clamp(R), channel decisions
    for (int v = t; v < g.n; v += NT) {
      const float x = F64 ? (float)llr64[base + v] : llr32[base + v];
      post[base + v] = x;
      int p0, dv;
      var_range<DV>(g, v, p0, dv);
      const float mx = v2c_store(x, x <= 0.0f);
      for (int j = 0; j < dv; ++j) *(float *)((char *)X + g.var_xoff[p0 + j]) = mx;
    }
    lds_barrier();

    int it = 0;
    for (;;) {
      uint32_t sxs = 0;  // OR of the checks' parities: bit 30 set iff one is unsatisfied
      if constexpr (DC > 0) {
        // two low-degree checks in flight per thread (more independent work per wave;
        // the higher degrees would lose resident waves to the registers it takes)
        constexpr int kCheckUnroll = DC <= 8 ? 2 : 1;
#pragma unroll kCheckUnroll
        for (int c = t; c < g.m; c += NT) {  // whole rows move with 8- or 16-byte LDS accesses
          float mv[DCM], ev[DCM];
          lds_row_load<DC>(X + c * DC, DC, mv);
          sxs |= check_core<DC, true>(mv, DC, ev);
          lds_row_store<DC>(X + c * DC, DC, ev);
        }
      } else {
        // one check per slot (a multiple of 64 slots; empty ones have degree 0), in place
        // on its interleaved row, which also holds half of the prefix pairs; whole groups
        // of 64 slots, one per wavefront pass, taken from the check phase's counter
        if (t == 0) s_next[1] = 0;
        for (int k = next_group(s_next); k < (xslots >> 6); k = next_group(s_next)) {
          const int sl = (k << 6) | (t & 63);
          const uint32_t info = (uint32_t)xslot[sl];
          const int dc = (int)(info >> 16);
          float *row = X + (info & 0xffffu);
          // one degree across the wavefront (every group of a quasi-cyclic code): the
          // code compiled for that degree, free of per-entry degree tests
          const int dcu = __builtin_amdgcn_readfirstlane(dc);
          if (__ballot(dc != dcu) == 0ull) {
            sxs |= check_core_row_uniform<DC, 64>(row, dcu);
          } else if (dc) {
            sxs |= check_core_row<DC, 64>(row, dc);
          }
        }
      }
      const unsigned long long b = __ballot(syndrome_bit(sxs));
      if ((t & 63) == 0) s_unsat[wave] = b != 0ull;
      lds_barrier();
      int any_unsat = 0;
      for (int w = 0; w < W; ++w) any_unsat |= s_unsat[w];
      if ((early_stop && !any_unsat) || it == max_iters) break;  // same value in every thread
      // The global reads of a variable (its edge list as LDS byte offsets, its channel
      // LLR) are issued ahead of its update (two variables ahead for the low fixed
      // degrees, one otherwise), so their latency overlaps the work on the ones before.
      // Register sets rotate (variables are taken in threes or pairs), so no loaded
      // value has to be copied out of the way of the next load.
      const float *__restrict__ lrow32 = llr32 + base;
      const double *__restrict__ lrow64 = llr64 + base;
      float *__restrict__ prow = post + base;
      // A variable's edge offsets: byte offsets for fixed degrees; for runtime degrees the
      // LDS float indices (< 2^16) two to a register, which leaves room for a third set.
      constexpr int kOffRegs = DV > 0 ? DVM : (DVM + 1) / 2;
      struct VarIn {
        int off[kOffRegs];
        int dv;
        float r;
      };
      auto offj = [](const VarIn &f, int j) -> int {
        if constexpr (DV > 0)
          return f.off[j];
        else
          return (int)((((uint32_t)f.off[j >> 1]) >> ((j & 1) << 4)) & 0xffffu) << 2;
      };
      // (32-bit byte offsets from uniform bases: the loads take an SGPR base address)
      auto fetch = [&](int vv, VarIn &f) {  // fixed degrees
        if constexpr (DV > 0) {
          int p0;
          var_range<DV>(g, vv, p0, f.dv);
          f.r = F64 ? (float)*(const double *)((const char *)lrow64 + (uint32_t)vv * 8u)
                    : *(const float *)((const char *)lrow32 + (uint32_t)vv * 4u);
          const int32_t *__restrict__ ve =
              (const int32_t *)((const char *)g.var_xoff + __umul24((uint32_t)vv, 4u * DVM));
#pragma unroll
          for (int j = 0; j < DVM; ++j) f.off[j] = ve[j];
        }
      };
      // X is the kernel's only LDS, so it starts at LDS address 0 (checked on the host)
      // and an edge's byte offset is its LDS address.
      auto xat = [](int off) { return (__attribute__((address_space(3))) float *)(size_t)off; };
      auto update_dv = [&](int v, const VarIn &f, int dv) __attribute__((always_inline)) {
        float ev[DVM];
#pragma unroll
        for (int j = 0; j < DVM; ++j)
          if (DV > 0 || j < dv) ev[j] = *xat(offj(f, j));
        const double L = var_total<DV>(f.r, ev, dv);
        const float Lf = (float)L;
        *(float *)((char *)prow + (uint32_t)v * 4u) = Lf;
        const bool z = Lf <= 0.0f;
#pragma unroll
        for (int j = 0; j < DVM; ++j)
          if (DV > 0 || j < dv) *xat(offj(f, j)) = v2c_store(var_extrinsic(L, ev[j]), z);
      };
      auto update = [&](int v, const VarIn &f) {
        if constexpr (DV > 0) {
          update_dv(v, f, DV);
        } else {  // one degree across the active lanes (a circulant's columns): the code
                  // compiled for that degree
          const int dvu = __builtin_amdgcn_readfirstlane(f.dv);
          if (__ballot(f.dv != dvu) == 0ull) {
            switch (dvu) {
#define LDPC_VAR_CASE(D)                      \
  case D:                                     \
    if constexpr (D <= DVM) update_dv(v, f, D); \
    break;
              LDPC_VAR_CASE(1) LDPC_VAR_CASE(2) LDPC_VAR_CASE(3) LDPC_VAR_CASE(4) LDPC_VAR_CASE(5)
              LDPC_VAR_CASE(6) LDPC_VAR_CASE(7) LDPC_VAR_CASE(8) LDPC_VAR_CASE(9) LDPC_VAR_CASE(10)
              LDPC_VAR_CASE(11) LDPC_VAR_CASE(12) LDPC_VAR_CASE(13) LDPC_VAR_CASE(14) LDPC_VAR_CASE(15)
              LDPC_VAR_CASE(16)
#undef LDPC_VAR_CASE
              default:
                update_dv(v, f, dvu);  // degree 0: the posterior is the channel value
                break;
            }
          } else {
            update_dv(v, f, f.dv);
          }
        }
      };
      const int vlast = g.n - 1;
      // low fixed degrees: three register sets, the reads two variables ahead (the
      // higher degrees' sets would cost them resident waves)
      if constexpr (DV > 0 && DV <= 3 && DC > 0 && DC <= 6) {
        VarIn fa, fb, fc;
        if (t < g.n) fetch(t, fa);
        if (t + NT < g.n) fetch(t + NT, fb);
        int v = t;
        for (; v + 2 * NT < g.n; v += 3 * NT) {
          fetch(v + 2 * NT, fc);
          update(v, fa);
          fetch(min(v + 3 * NT, vlast), fa);
          update(v + NT, fb);
          fetch(min(v + 4 * NT, vlast), fb);
          update(v + 2 * NT, fc);
        }
        if (v < g.n) update(v, fa);
        if (v + NT < g.n) update(v + NT, fb);
      } else if constexpr (DV < 0) {
        // groups of 64 variables from the variable phase's counter, in the order of the
        // table after the check slots; the reads of the next group are issued before the
        // update of the current one (two register sets: a third one of up to 16 offsets
        // would spill)
        if (t == 0) s_next[0] = 0;
        // (position k of the order holds the group's index, where its rows start in the
        // table and its degree when all its variables share one, else -1; the rows are the
        // 64 lanes' degrees, then entry j of every lane's edge offsets, each read by the
        // wavefront as one contiguous 256-byte segment)
        const int32_t *__restrict__ vorder = xslot + xslots;
        const int vgroups = (g.n + 63) >> 6;
        auto fetch_group = [&](int k, int &v, VarIn &f) {
          v = (ld_graph(vorder, (size_t)3 * k) << 6) | (t & 63);
          if (v >= g.n) return;
          const int32_t *__restrict__ ve = xslot + ld_graph(vorder, (size_t)3 * k + 1) + (t & 63);
          const int ud = ld_graph(vorder, (size_t)3 * k + 2);
          f.dv = ud >= 0 ? ud : ve[0];
          f.r = F64 ? (float)*(const double *)((const char *)lrow64 + (uint32_t)v * 8u)
                    : *(const float *)((const char *)lrow32 + (uint32_t)v * 4u);
#pragma unroll
          for (int r = 0; r < kOffRegs; ++r)
            if (2 * r < f.dv) f.off[r] = ve[(r + 1) << 6];
        };
        VarIn fa, fb, fc;
        int ka = next_group(s_next + 1), va = 0, vb = 0, vc = 0;
        if (ka < vgroups) fetch_group(ka, va, fa);
        int kb = next_group(s_next + 1);
        if (kb < vgroups) fetch_group(kb, vb, fb);
        while (ka < vgroups) {
          const int kc = next_group(s_next + 1);
          if (kc < vgroups) fetch_group(kc, vc, fc);
          if (va < g.n) update(va, fa);
          if (kb >= vgroups) break;
          ka = next_group(s_next + 1);
          if (ka < vgroups) fetch_group(ka, va, fa);
          if (vb < g.n) update(vb, fb);
          if (kc >= vgroups) break;
          kb = next_group(s_next + 1);
          if (kb < vgroups) fetch_group(kb, vb, fb);
          if (vc < g.n) update(vc, fc);
        }
      } else {
        // two sets (the higher fixed degrees would lose resident waves to a third)
        VarIn fa, fb;
        if (t < g.n) fetch(t, fa);
        int v = t;
        for (; v + NT < g.n; v += 2 * NT) {
          fetch(v + NT, fb);
          update(v, fa);
          fetch(min(v + 2 * NT, vlast), fa);
          update(v + NT, fb);
        }
        if (v < g.n) update(v, fa);
      }
      lds_barrier();  // also orders this iteration's reads of s_unsat before the next writes
      ++it;
    }

    for (int v = t; v < g.n; v += NT) hard[base + v] = post[base + v] <= 0.0f ? 1 : 0;  // own writes
    if (t == 0) iters[word] = it;
    lds_barrier();  // X, s_word and s_unsat are reused by the next word
  }
}

__global__ void reset_counter(int *counter) {
  if (threadIdx.x == 0) *counter = 0;
}

}  // namespace ldpc

using namespace ldpc;

namespace {
using StreamKernel = void (*)(GraphDev, const float *, const double *, int, int, int, int *, uint8_t *, float *,
                              int32_t *, const int32_t *, int, int);

// The kernel for a graph's degrees and the LLR precision (FP32 or FP64 input).
StreamKernel pick_stream(const ldpc_graph_s *g, int &max_threads, bool f64 = false) {
  StreamKernel k = nullptr;
#define LDPC_PICK(C, V)                                                          \
  k = f64 ? stream_decode_kernel<C, V, true> : stream_decode_kernel<C, V, false>; \
  max_threads = kStreamMaxThreads<C>
  LDPC_KIND_SWITCH(kernel_kind(g), LDPC_PICK)
#undef LDPC_PICK
  return k;
}

// Default workgroup size: the one that keeps the most threads resident per compute
// unit (LDS and registers both limit it), from 64 up to the power of two covering the
// larger of m and n but not above 512; on a tie the larger workgroup.  A batch smaller
// than the resident capacity is counted at its own size.  Above 512 threads the cost
// of bringing every wave to each of the two barriers per iteration outweighs the
// shorter phases: 512 beat 1024 on (3,6) n=4096 both in throughput (by ~5 %) and for
// a single word, and on the n=1032 Table I codes.  The exception is a word state so
// large that one workgroup fills a compute unit's LDS: then 8 waves cannot hide the
// LDS and memory latencies and 1024 threads (16 waves) are taken when they fit.
constexpr int kStreamDefaultMaxThreads = 512;

int stream_threads(const ldpc_graph_s *g, int max_threads, int32_t batch) {
  const int big = std::max(g->m, g->n);
  const int cap = std::min(max_threads, kStreamDefaultMaxThreads);
  int top = 64;
  while (top < cap && top < big) top *= 2;
  int best_nt = 0;
  long best = -1;
  for (int i = 4; i >= 0; --i) {
    const int nt = 64 << i;
    if (nt > top || g->stream_per_cu[i] < 1) continue;
    const long groups = std::min<long>((long)g->stream_per_cu[i] * g->stream_cus, batch);
    if (groups * nt > best) {
      best = groups * nt;
      best_nt = nt;
    }
  }
  if (max_threads >= 1024 && top >= kStreamDefaultMaxThreads && big > kStreamDefaultMaxThreads &&
      g->stream_per_cu[4] >= 1 && g->stream_per_cu[3] <= 1)
    best_nt = 1024;
  return best_nt;
}

// Device facts the launch needs (the LDS opt-in of the kernel, compute units, resident
// workgroups per size) and the LDS placement of the rows, prepared once per graph.
ldpc_status stream_prepare(ldpc_graph_s *g, StreamKernel k, int max_threads, size_t lds) {
  std::lock_guard<std::mutex> lock(g->stream_mu);
  if (g->stream_ready) return LDPC_OK;
  int dev = 0, cus = 0, lim = 0;
  LDPC_HIP_CHECK(hipGetDevice(&dev));
  LDPC_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  LDPC_HIP_CHECK(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  g->stream_lds_limit = lim;
  if (lds + 64 <= (size_t)lim) {
    std::vector<int32_t> off;
    if (kernel_kind(g) < KIND_G8) {
      off = stream_edge_offsets(g);
    } else {
      const StreamGroupLayout L = stream_group_layout(g);
      if (L.floats != g->stream_x_floats)  // the size the LDS was sized with
        return set_error(LDPC_ERR_DEVICE, "stream layout size disagrees with the graph's LDS size");
      off.resize((size_t)g->nnz);
      for (size_t p = 0; p < off.size(); ++p) off[p] = L.pos[(size_t)g->var_edges[p]] * 4;
      const std::vector<int32_t> tab = stream_group_table(g, L, off);
      if (!g->d_xslot) {
        LDPC_HIP_CHECK(hipMalloc((void **)&g->d_xslot, tab.size() * sizeof(int32_t)));
        g->stream_slots = (int32_t)L.slot.size();
      }
      LDPC_HIP_CHECK(hipMemcpy(g->d_xslot, tab.data(), tab.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    LDPC_HIP_CHECK(hipMemcpy(g->d_var_xoff, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  }
  if (lds + 64 > (size_t)lim) {  // cannot run; remember the limit only
    g->stream_cus = cus;
    g->stream_ready = true;
    return LDPC_OK;
  }
  LDPC_HIP_CHECK(hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipFuncAttributes fa{};
  LDPC_HIP_CHECK(hipFuncGetAttributes(&fa, (const void *)k));
  if (fa.sharedSizeBytes != 0)  // the kernel addresses its messages from LDS address 0
    return set_error(LDPC_ERR_DEVICE, "stream kernel has static LDS; its message array would not start at 0");
  int mt = 0;
  StreamKernel k64 = pick_stream(g, mt, true);
  LDPC_HIP_CHECK(hipFuncSetAttribute((const void *)k64, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  LDPC_HIP_CHECK(hipFuncGetAttributes(&fa, (const void *)k64));
  if (fa.sharedSizeBytes != 0)
    return set_error(LDPC_ERR_DEVICE, "stream kernel has static LDS; its message array would not start at 0");
  for (int i = 0; i < 5; ++i) {
    const int nt = 64 << i;
    int per_cu = 0;
    if (nt <= max_threads)
      LDPC_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k, nt, lds));
    g->stream_per_cu[i] = per_cu;
  }
  g->stream_cus = cus;
  g->stream_ready = true;
  return LDPC_OK;
}
}  // namespace

extern "C" ldpc_status ldpc_stream_lds_bytes(ldpc_graph_t g, size_t *bytes, int32_t *supported) {
  if (!g) return set_error(LDPC_ERR_INVALID_ARG, "graph is NULL");
  const size_t b = stream_lds_bytes(g);
  if (bytes) *bytes = b;
  if (supported) {
    int dev = 0, lim = 0;
    LDPC_HIP_CHECK(hipGetDevice(&dev));
    LDPC_HIP_CHECK(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    *supported = b + 64 <= (size_t)lim ? 1 : 0;
  }
  return LDPC_OK;
}

ldpc_status stream_ready_for(ldpc_graph_s *g, int32_t threads) {
  int max_threads = 1024;
  StreamKernel k = pick_stream(g, max_threads);
  if (threads > max_threads)
    return set_error(LDPC_ERR_INVALID_ARG,
                     "threads above " + std::to_string(max_threads) + " for this code's check degree");
  const size_t lds = stream_lds_bytes(g);
  ldpc_status st = stream_prepare(g, k, max_threads, lds);
  if (st != LDPC_OK) return st;
  if (lds + 64 > (size_t)g->stream_lds_limit)
    return set_error(LDPC_ERR_UNSUPPORTED, "word state (" + std::to_string(lds) + " bytes) exceeds LDS");
  return LDPC_OK;
}

ldpc_status launch_stream_decode(ldpc_graph_s *g, const void *llr, bool llr_f64, int32_t batch, int32_t max_iters,
                                 int32_t early_stop, uint8_t *hard_bits, float *posterior, int32_t *iters_used,
                                 int *counter, int32_t threads, hipStream_t stream) {
  ldpc_status st = stream_ready_for(g, threads);
  if (st != LDPC_OK) return st;
  if (batch == 0) return LDPC_OK;
  int max_threads = 1024;
  StreamKernel k = pick_stream(g, max_threads, llr_f64);
  const size_t lds = stream_lds_bytes(g);
  const int nt = threads ? threads : stream_threads(g, max_threads, batch);
  if (nt == 0) return set_error(LDPC_ERR_UNSUPPORTED, "stream kernel cannot be resident");
  int per_cu = 0;
  if ((nt & (nt - 1)) == 0) {  // powers of two: resident counts known
    int lg = 0;
    while ((64 << lg) < nt) ++lg;
    per_cu = g->stream_per_cu[lg];
  } else {
    LDPC_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k, nt, lds));
  }
  if (per_cu < 1) return set_error(LDPC_ERR_UNSUPPORTED, "stream kernel cannot be resident");
  const int grid = std::min(batch, g->stream_cus * per_cu);
  hipLaunchKernelGGL(reset_counter, dim3(1), dim3(64), 0, stream, counter);
  LDPC_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k, dim3(grid), dim3(nt), lds, stream, graph_dev(g),
                     llr_f64 ? nullptr : (const float *)llr, llr_f64 ? (const double *)llr : nullptr, (int)batch,
                     (int)max_iters, (int)(early_stop != 0), counter, hard_bits, posterior, iters_used,
                     (const int32_t *)g->d_xslot, (int)g->stream_slots, (int)stream_x_bytes(g));
  LDPC_HIP_CHECK(hipGetLastError());
  return LDPC_OK;
}

extern "C" ldpc_status ldpc_decode_stream(ldpc_graph_t g, const void *llr, int32_t batch, int32_t max_iters,
                                          int32_t early_stop, uint32_t flags, uint8_t *hard_bits, float *posterior,
                                          int32_t *iters_used, void *workspace, size_t ws_bytes, int32_t threads,
                                          hipStream_t stream) {
  if (!g) return set_error(LDPC_ERR_INVALID_ARG, "graph is NULL");
  if (batch < 0 || max_iters < 0) return set_error(LDPC_ERR_INVALID_ARG, "negative batch or max_iters");
  if (flags & ~LDPC_LLR_F64) return set_error(LDPC_ERR_INVALID_ARG, "unknown flag");
  if (threads != 0 && (threads < 64 || threads > 1024 || threads % 64))
    return set_error(LDPC_ERR_INVALID_ARG, "threads must be 0 or a multiple of 64 in 64..1024");
  if (batch == 0) return LDPC_OK;
  if (!llr || !hard_bits || !posterior || !iters_used || !workspace)
    return set_error(LDPC_ERR_INVALID_ARG, "NULL buffer");
  if (ws_bytes < 256) return set_error(LDPC_ERR_INVALID_ARG, "workspace too small (256 bytes)");
  return launch_stream_decode(g, llr, (flags & LDPC_LLR_F64) != 0, batch, max_iters, early_stop, hard_bits, posterior,
                              iters_used, (int *)workspace, threads, stream);
}
