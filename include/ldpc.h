/*
 * ldpc.h -- C ABI of the MI355X flooding sum-product LDPC decoder.
 *
 * The operation is the sum-product (belief-propagation) decoding of a binary
 * LDPC code of Sec. II-B (Eqs. 4-8) in the flooding order of Algorithm 1 (all
 * check nodes, then all variable nodes, per iteration), applied independently to
 * a batch of received words: the "batch processing" decomposition of Sec. III-C,
 * where every worker decodes whole words.  A syndrome test (H z^T = 0, Eq. 1)
 * may end each word early.
 *
 * Conventions shared by every entry point
 *  - batch (words per call) is at most 2^31 - 64: tile counts are (batch + 63) / 64 in
 *    32-bit arithmetic.  Split larger batches into several calls.
 *  - H is m x n.  Edges are numbered in CSR order: check-major, variables
 *    ascending inside a check.  Per-edge arrays (weights, gradients) use it.
 *  - LLRs are log P(c=0)/P(c=1) (BPSK x = 1 - 2c gives lambda = 2y/sigma^2,
 *    Eq. 4 with the ratio inverted); decisions are z_v = 1 iff L_v <= 0 (Eq. 8
 *    for this sign).  With this sign the check rule of Eq. 5 holds for every
 *    check degree.
 *  - Check rule (Eq. 5, denominator 1 - prod): E_cv = 2 atanh(prod_{v'!=v} tanh(M_v'c/2)),
 *    evaluated as ln(s/d) of the pair d = (A-B)/2, s = (A+B)/2 with A = prod(1+q),
 *    B = prod(1-q), q = e^-|M| over the other messages (exclusive prefix and suffix
 *    pairs, joined in FP64), the sign as the parity of the others.  Messages and
 *    posteriors are stored in FP32.
 *  - Variable rule (Eq. 6): M_vc = clamp(R_v + sum_{c'!=c} E_c'v, -20, 20); posterior
 *    (Eq. 7) L_v = R_v + sum_c E_cv (ascending check order); both summed in FP64 and
 *    rounded once to FP32.
 *  - Messages start at E = 0, so the first check update sees M = clamp(R).
 *  - Device pointers are device memory owned by the caller; host pointers are
 *    read during the call only.  Work is enqueued on the given HIP stream and the
 *    call returns without waiting.  Nothing throws across this boundary: every
 *    entry point returns an ldpc_status; ldpc_last_error() gives the detail of
 *    the calling thread's last failure.
 */
#ifndef LDPC_H
#define LDPC_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LDPC_OK = 0,
  LDPC_ERR_INVALID_ARG = -1,   /* null pointer, negative size, short workspace, bad flag */
  LDPC_ERR_BAD_MATRIX = -2,    /* malformed H (see ldpc_graph_create) */
  LDPC_ERR_OUT_OF_MEMORY = -3, /* host or device allocation failed */
  LDPC_ERR_DEVICE = -4,        /* a HIP call failed (detail in ldpc_last_error) */
  LDPC_ERR_UNSUPPORTED = -5    /* degree above the kernel limits */
} ldpc_status;

typedef enum {
  LDPC_CSR = 0, /* ptr has m+1 entries over checks, idx holds variable indices */
  LDPC_CSC = 1  /* ptr has n+1 entries over variables, idx holds check indices */
} ldpc_format;

/* Largest check and variable degrees the kernels accept. */
#define LDPC_MAX_CHECK_DEGREE 32
#define LDPC_MAX_VAR_DEGREE 16

/* flags of ldpc_decode / ldpc_decode_workspace_size */
#define LDPC_LLR_F64 0x1u /* llr is double [batch][n]; rounded to FP32 once on ingest */

typedef struct ldpc_graph_s *ldpc_graph_t;

/*
 * Tanner graph of H (Sec. II-B: an edge joins check c and variable v for every
 * 1 in H[c][v]; Fig. 1).  ptr/idx are host arrays, copied; nnz = ptr[last].
 * Returns LDPC_ERR_BAD_MATRIX if m or n <= 0, ptr is not non-decreasing from 0
 * to nnz, an index is out of range, an entry is repeated, or a check has degree
 * < 2; LDPC_ERR_UNSUPPORTED if a degree exceeds the limits above.  Variables of
 * degree 0 are allowed (their posterior is the channel LLR).  The graph holds
 * device copies of its index arrays on the current device until destroyed and
 * must outlive the work enqueued with it.
 */
ldpc_status ldpc_graph_create(int32_t m, int32_t n, ldpc_format fmt, const int32_t *ptr, const int32_t *idx,
                              int64_t nnz, ldpc_graph_t *out);
ldpc_status ldpc_graph_destroy(ldpc_graph_t g);

/* Sizes and degree extremes; any output pointer may be NULL. */
ldpc_status ldpc_graph_info(ldpc_graph_t g, int32_t *m, int32_t *n, int64_t *edges, int32_t *max_check_deg,
                            int32_t *max_var_deg);

/* Host copies of the edge numbering: check_of_edge[e], var_of_edge[e] for e < edges (either may be NULL). */
ldpc_status ldpc_graph_edges(ldpc_graph_t g, int32_t *check_of_edge, int32_t *var_of_edge);

/* Device workspace bytes for ldpc_decode at full speed on the current device: 256 bytes plus
 * one 64-word tile state (the messages of 64 words) per workgroup the device holds resident at
 * once with ldpc_decode's launch shape, at most one per tile of the batch.  Workgroups take
 * tiles from a counter and reuse their tile state, so a smaller workspace (at least 256 bytes
 * plus one tile state) also works, with fewer tiles in flight. */
ldpc_status ldpc_decode_workspace_size(ldpc_graph_t g, int32_t batch, uint32_t flags, size_t *bytes);

/*
 * Plain flooding decode of `batch` words (Sec. II-B, Eqs. 4-8; batch split of
 * Sec. III-C).  llr: device [batch][n], FP32 (or FP64 with LDPC_LLR_F64).
 * Outputs (device, [batch][n] / [batch]): hard_bits 0/1, posterior L_v (FP32),
 * iters_used.  With early_stop != 0 a word stops at the first t in 0..max_iters
 * whose decisions satisfy H z^T = 0 (t = 0 tests the channel decisions); its
 * outputs are those of iteration t.  Otherwise every word runs max_iters.
 * max_iters = 0 returns the channel LLRs.  batch = 0 is a no-op.
 * workspace: device, 256-byte aligned, ldpc_decode_workspace_size bytes for full speed and
 * at least 256 bytes plus one tile state (LDPC_ERR_INVALID_ARG below that); its contents need
 * no initialisation and are garbage afterwards.
 */
ldpc_status ldpc_decode(ldpc_graph_t g, const void *llr, int32_t batch, int32_t max_iters, int32_t early_stop,
                        uint32_t flags, uint8_t *hard_bits, float *posterior, int32_t *iters_used, void *workspace,
                        size_t ws_bytes, hipStream_t stream);

/*
 * ldpc_decode with the c->v state in and out (one-step checks of Eqs. 5-7 from a given
 * state; resuming a decode).  init_cv: NULL, or device [batch][edges] FP32 c->v messages
 * E^(0) in CSR edge order to start from instead of zeros.  Then the iteration-0 posterior
 * is L^(0) = R + sum_c E^(0)_cv (Eq. 7 on that state, ascending check order), its
 * decisions are tested first when early_stop is set (a word that stops there returns
 * L^(0) and its decisions), and iteration 1 forms M^(1) = clamp(R + sum_{c'!=c} E^(0)_c'v)
 * (Eq. 6).  final_cv: NULL, or device [batch][edges]: receives each word's c->v messages
 * of its last iteration, E^(iters_used) (init_cv, or zeros without it, for a word that
 * stops at 0).  With both NULL this is ldpc_decode; otherwise the same arguments, the
 * same workspace and the same errors, plus LDPC_ERR_INVALID_ARG for a state pointer on
 * a graph without edges.  The buffers are read or written only during the enqueued work.
 */
ldpc_status ldpc_decode_ex(ldpc_graph_t g, const void *llr, int32_t batch, int32_t max_iters, int32_t early_stop,
                           uint32_t flags, const float *init_cv, float *final_cv, uint8_t *hard_bits,
                           float *posterior, int32_t *iters_used, void *workspace, size_t ws_bytes,
                           hipStream_t stream);

/*
 * ldpc_decode without any allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid it): the
 * tile state lives in a fixed device array of LDPC_NOALLOC_SCRATCH_BYTES that the
 * library holds on each GPU it runs on until the process ends.  Same arguments (minus
 * the workspace), outputs (bit for bit), and errors as ldpc_decode, plus
 * LDPC_ERR_INVALID_ARG when the workspace ldpc_decode would take at full speed
 * (ldpc_decode_workspace_size) exceeds the array: for codes whose resident workgroups' tile
 * states fill more than the array, at most floor((LDPC_NOALLOC_SCRATCH_BYTES - 256) / tile
 * bytes) x 64 words per call (384 words of a (3,6) n=4096 code, 17 472 of an n=96 code); any
 * batch of a code small enough that they do not.  The first call on
 * a device looks up that device's copy of the array (hipGetSymbolAddress); no call
 * allocates or frees memory.  Every call on a GPU uses the same array: calls that
 * overlap on one GPU (different streams, or different threads) race and must be
 * serialised by the caller.  The array needs no clearing between calls.
 */
#define LDPC_NOALLOC_SCRATCH_BYTES (64u << 20)
ldpc_status ldpc_decode_noalloc(ldpc_graph_t g, const void *llr, int32_t batch, int32_t max_iters,
                                int32_t early_stop, uint32_t flags, uint8_t *hard_bits, float *posterior,
                                int32_t *iters_used, hipStream_t stream);

/* Decode with an explicit launch shape: waves per workgroup (1..16; ldpc_decode uses 16).
 * Same contract as ldpc_decode. */
ldpc_status ldpc_decode_config(ldpc_graph_t g, const void *llr, int32_t batch, int32_t max_iters, int32_t early_stop,
                               uint32_t flags, uint8_t *hard_bits, float *posterior, int32_t *iters_used,
                               void *workspace, size_t ws_bytes, int32_t waves, hipStream_t stream);

/* ---- stream form: one word per workgroup, state in LDS -------------------- */

/* LDS bytes one word's decoding state needs and whether it fits one workgroup of the current
 * device (*supported = 1).  The state is one FP32 message per edge plus 80 bytes, the message
 * array rounded up to 16 bytes.  Codes outside the fixed degree pairs interleave the rows of 64
 * checks at a time (the checks sorted by degree, ties by index); such a group spans 64 x its
 * largest degree floats, the last group only up to its last entry, so the array exceeds the
 * edge count only where a group mixes degrees.  *supported may be NULL (then no device is
 * queried). */
ldpc_status ldpc_stream_lds_bytes(ldpc_graph_t g, size_t *bytes, int32_t *supported);

/*
 * Same contract and bit-identical outputs as ldpc_decode, computed by the stream
 * form (Sec. III-B's spreading of one word over many workers, here the threads of
 * one workgroup with every message in LDS).  Persistent workgroups take words from
 * an atomic counter.  threads: workgroup size (multiple of 64 up to 1024; 0 = the
 * size up to 512 that keeps the most threads resident, or 1024 when one 512-thread
 * workgroup fills a compute unit's LDS); another value returns LDPC_ERR_INVALID_ARG.  The channel LLRs are read again in every iteration.  workspace: >= 256 device
 * bytes (the counter).  Returns LDPC_ERR_UNSUPPORTED when the word state exceeds the
 * LDS of one workgroup.
 */
ldpc_status ldpc_decode_stream(ldpc_graph_t g, const void *llr, int32_t batch, int32_t max_iters, int32_t early_stop,
                               uint32_t flags, uint8_t *hard_bits, float *posterior, int32_t *iters_used,
                               void *workspace, size_t ws_bytes, int32_t threads, hipStream_t stream);

/* ---- split form: each half-iteration a launch over many workgroups per tile -- */

/*
 * Same contract and bit-identical outputs as ldpc_decode, for batches with few
 * 64-word tiles: the plain decoder gives a tile one workgroup for the whole decode,
 * here each check phase and each variable phase of Algorithm 1 is its own launch
 * that spreads every tile's checks (variables) over `slices` workgroups (0 = about
 * 2048 workgroups in all, at least 4 checks or variables per wave); the launch
 * boundary is the exchange between the phases.  2 (max_iters + 1) + 2 launches are
 * enqueued; tiles whose words have all stopped return at once.  workspace: device,
 * >= ldpc_split_workspace_size bytes, 256-byte aligned, no initialisation needed.
 */
ldpc_status ldpc_split_workspace_size(ldpc_graph_t g, int32_t batch, size_t *bytes);
ldpc_status ldpc_decode_split(ldpc_graph_t g, const void *llr, int32_t batch, int32_t max_iters, int32_t early_stop,
                              uint32_t flags, uint8_t *hard_bits, float *posterior, int32_t *iters_used,
                              void *workspace, size_t ws_bytes, int32_t slices, hipStream_t stream);

/* ---- batched persistent form --------------------------------------------- */

/* Most codes one batched launch serves. */
#define LDPC_MAX_CODES 8

/* One code's share of a batched decode; all pointers are device memory. */
typedef struct {
  const float *llr;   /* [batch][n] FP32 channel LLRs */
  int32_t batch;      /* words of this code (>= 0) */
  int32_t max_iters;  /* iteration limit of this code (>= 0) */
  uint8_t *hard_bits; /* [batch][n] out */
  float *posterior;   /* [batch][n] out */
  int32_t *iters_used;/* [batch] out */
} ldpc_job;

/* Launch shape of a batched decode: waves per workgroup (0 = 16 when the batch has
 * fewer 64-word tiles than the GPU has compute units, else 8); 64-word slots
 * (workgroups) per code (0 = automatic: the resident capacity of the GPU shared
 * in proportion to words x edges, at most one slot per 64 words); refill: a slot
 * writes out and replaces its stopped words once this many of its 64 lanes wait
 * (0 = 1), or when none is still running.  stream_codes: bit q set = code q is
 * decoded by the stream form instead (one word per workgroup, state in LDS, its own
 * launch before the persistent one; same outputs bit for bit; the code's word
 * state must fit, see ldpc_stream_lds_bytes, else LDPC_ERR_UNSUPPORTED);
 * LDPC_STREAM_AUTO = every code whose word state fits; 0 = none. */
#define LDPC_STREAM_AUTO 0xFFFFFFFFu
/* split_codes: bit q set = code q (if not in stream form) is decoded by the split form
 * (ldpc_decode_split, its own launches before the persistent one; same outputs bit for
 * bit); LDPC_SPLIT_AUTO = every such code whose words fill fewer 64-word tiles than
 * half the GPU's compute units; 0 = none. */
#define LDPC_SPLIT_AUTO 0xFFFFFFFFu
/* lanes: words one slot holds at a time (1..64; 0 = 64); a code has at most ceil(batch / lanes)
 * slots, and at most as many as the GPU holds resident at once (slots beyond that would start
 * only when the code's queue is empty).
 * stream_threads[q]: workgroup size of code q in the stream form (0 = automatic, else as
 * ldpc_decode_stream's threads); split_slices[q]: workgroups per tile of code q in the split
 * form (0 = automatic, else as ldpc_decode_split's slices).
 * span[q]: workgroups that share each slot of code q (1..64; 0 = automatic: 1, or, when the
 * code's slot count is automatic and its words fill fewer slots than its share of the resident
 * capacity, that share divided by its slots).  A slot of span > 1 ("group slot") splits every
 * check and variable phase over its workgroups, which meet at a barrier in global memory after
 * each phase: a batch with few words of a long code then keeps many compute units busy.  Its
 * workgroups wait for each other, so a launch with group slots must fit the GPU at once:
 * sum over codes of slots x span <= resident workgroups of the kernel (automatic spans shrink to
 * fit; explicit ones that do not fit are LDPC_ERR_INVALID_ARG).  The barrier gives up after
 * seconds of waiting (possible only if other work keeps the launch's workgroups from becoming
 * resident that long; the environment variable LDPC_GROUP_SPIN_LIMIT, read at each launch, sets
 * the number of polls instead, for tests of this path); the int at byte offset
 * LDPC_MULTI_FAULT_OFFSET of the workspace is then nonzero after the launch, and its outputs are
 * invalid. */
typedef struct {
  int32_t waves;
  int32_t slots[LDPC_MAX_CODES];
  int32_t refill;
  uint32_t stream_codes;
  uint32_t split_codes;
  int32_t lanes;
  int32_t stream_threads[LDPC_MAX_CODES];
  int32_t split_slices[LDPC_MAX_CODES];
  int32_t span[LDPC_MAX_CODES];
} ldpc_multi_shape;
#define LDPC_MULTI_FAULT_OFFSET 480

/* Shape ldpc_decode_multi would use (automatic slot counts, the stream and split masks
 * filled in; codes in stream or split form get 0 slots) and its workspace size. */
ldpc_status ldpc_multi_resolve(const ldpc_graph_t *graphs, int32_t ncodes, const ldpc_job *jobs,
                               const ldpc_multi_shape *shape, ldpc_multi_shape *resolved, size_t *ws_bytes);

/*
 * Batched decode of the words of up to LDPC_MAX_CODES codes in one persistent
 * launch (the batch processing of Sec. III-C with a shared work queue).  Each
 * 64-lane slot holds words of one code; a word that stops (the syndrome test of
 * Eq. 1 with early_stop, or its code's max_iters) writes its outputs and its lane
 * takes the next word of that code.  Per word the arithmetic and the outputs are
 * identical (bit for bit) to ldpc_decode with the same early_stop and max_iters.
 * orders: NULL, or per code NULL or a device permutation of 0..batch-1 giving the
 * order in which words are taken (outputs stay at each word's own index).
 * workspace: device, >= ldpc_multi_resolve's size, 256-byte aligned; no
 * initialisation needed.  Enqueued on `stream`.
 */
ldpc_status ldpc_decode_multi(const ldpc_graph_t *graphs, int32_t ncodes, const ldpc_job *jobs,
                              const int32_t *const *orders, int32_t early_stop, const ldpc_multi_shape *shape,
                              void *workspace, size_t ws_bytes, hipStream_t stream);

/* A batched decode captured once into a HIP graph (fixed pointers and shapes) and replayed. */
typedef struct ldpc_plan_s *ldpc_plan_t;
/* Captures the launch sequence of ldpc_decode_multi on capture_stream (a non-default stream). */
ldpc_status ldpc_plan_create_multi(const ldpc_graph_t *graphs, int32_t ncodes, const ldpc_job *jobs,
                                   const int32_t *const *orders, int32_t early_stop, const ldpc_multi_shape *shape,
                                   void *workspace, size_t ws_bytes, hipStream_t capture_stream, ldpc_plan_t *out);
ldpc_status ldpc_plan_launch(ldpc_plan_t plan, hipStream_t stream);
ldpc_status ldpc_plan_destroy(ldpc_plan_t plan);

/*
 * Autotuner: times candidate shapes of this batched decode on the given inputs and
 * returns the fastest in *best (and its time in *best_ms).  Starting from the automatic
 * choice (stream form for the codes whose word state fits LDS, split form for the other
 * codes with few tiles, the persistent launch for the rest), it tries every other form
 * for one code at a time and keeps what is faster (one pass over the codes), then each
 * stream-form code's workgroup size and each split-form code's slices, then the
 * persistent launch's shape (waves per workgroup x slot scale x refill threshold x slot
 * width, and halved and quartered automatic spans) when a code uses it, then each persistent
 * code's span doubled and halved.  Candidates that the launch cannot take (group slots beyond
 * the resident capacity) are skipped.  Every candidate runs once to warm up and then 2 to 16 times
 * (about 40 ms in all); its time is the median.  The winner and the automatic start are timed
 * again at the end, and the start is returned unless the winner is more than 2 % faster.
 * Writes the jobs' outputs; allocates and frees its own temporary workspace (the largest
 * any candidate needs).  Synchronises `stream`.
 */
#define LDPC_TUNE_PERSISTENT_ONLY 0x1u /* flags: every code in the persistent launch; tune its shape only */
ldpc_status ldpc_autotune_multi(const ldpc_graph_t *graphs, int32_t ncodes, const ldpc_job *jobs,
                                const int32_t *const *orders, int32_t early_stop, uint32_t flags,
                                hipStream_t stream, ldpc_multi_shape *best, float *best_ms);

/* ---- differentiable form --------------------------------------------------- */

/*
 * Unrolled flooding decoder with a weight on every c->v message where it enters a
 * variable-node sum (Eqs. 5-7 with weights; T iterations, no early stop):
 *   A^(1)_e = R_v,  E^(t) = Eq. 5 on clamp(A^(t)),
 *   A^(t+1)_e = R_v + sum_{e' in N(v), e' != e} w[t-1][e'] E^(t)_e',
 *   L_v = R_v + sum_{e in N(v)} w[T-1][e] E^(T)_e.
 * All weights 1 gives ldpc_decode(early_stop = 0, max_iters = T) bit for bit.
 * Sizes: checkpoints (the A^(t) of every iteration, kept between forward and
 * backward), forward and backward workspaces, all device bytes, for this graph,
 * batch and T.  Their layout is internal: a code whose per-word backward state
 * (4 x edges + 4 x n bytes) fits the LDS of one workgroup runs one word per
 * workgroup with its messages on chip; larger codes run 64-word tiles in HBM.
 */
ldpc_status ldpc_unrolled_sizes(ldpc_graph_t g, int32_t batch, int32_t T, size_t *ckpt_bytes, size_t *fwd_ws_bytes,
                                size_t *bwd_ws_bytes);

/* llr [batch][n], w [T][edges] (edge order of ldpc_graph_edges), posterior [batch][n] out,
 * ckpt written (caller-owned, 256-byte aligned); all device, FP32. */
ldpc_status ldpc_unrolled_forward(ldpc_graph_t g, const float *llr, const float *w, int32_t batch, int32_t T,
                                  float *posterior, void *ckpt, size_t ckpt_bytes, void *workspace, size_t ws_bytes,
                                  hipStream_t stream);

/* Adjoint of ldpc_unrolled_forward: given d loss / d posterior [batch][n] and the
 * forward's checkpoints (unchanged), writes d loss / d llr [batch][n] and
 * d loss / d w [T][edges] (summed over the batch in a fixed order; deterministic).
 * Check-node messages are recomputed from the checkpoints. */
ldpc_status ldpc_unrolled_backward(ldpc_graph_t g, const float *w, const void *ckpt, size_t ckpt_bytes,
                                   const float *grad_post, int32_t batch, int32_t T, float *grad_llr, float *grad_w,
                                   void *workspace, size_t ws_bytes, hipStream_t stream);

/* ---- word generation: systematic encoder, BPSK/AWGN channel, error counts -- */

typedef struct ldpc_encoder_s *ldpc_encoder_t;

/*
 * Systematic encoder of the code of g.  Codewords are the words c with
 * H c^T = 0 (Eq. 1), the row space of a generator G, and a message m of k bits
 * is sent as c = m G (Eqs. 2-3); a systematic G copies m into k positions
 * (the [I_k : P] form of Sec. III-B up to a column permutation).  The
 * positions: H is reduced over GF(2) with pivot columns taken from the last
 * column towards the first (the first remaining row with a 1 in a column becomes
 * its pivot row); rank = number of pivots, k = n - rank; the non-pivot columns,
 * ascending, carry the message (message bit j goes to info[j]) and the pivot
 * column of reduced row r carries the parity of the message bits in that row.
 * The reduction runs on the host at create (bit-packed rows; seconds for
 * n ~ 16k).  The encoder holds device arrays on the current device (A: rank x
 * ceil(k/64) 64-bit words, a column map of n int32) until destroyed and is
 * independent of g afterwards.
 */
ldpc_status ldpc_encoder_create(ldpc_graph_t g, ldpc_encoder_t *out);
ldpc_status ldpc_encoder_destroy(ldpc_encoder_t e);
ldpc_status ldpc_encoder_info(ldpc_encoder_t e, int32_t *n, int32_t *k, int32_t *rank);
/* Host outputs (each may be NULL): info [k] message positions, pivots [rank] the
 * pivot column of reduced row r. */
ldpc_status ldpc_encoder_positions(ldpc_encoder_t e, int32_t *info, int32_t *pivots);

/*
 * Codewords of caller messages: msg [batch][k] bytes (any nonzero byte is a 1),
 * cw [batch][n] bytes 0/1 out, both device memory, cw 4-byte aligned.  One
 * workgroup per 64 words keeps their messages (64 x 8 ceil(k/64) bytes) and
 * parity bits (8 x rank bytes, rank rounded up to 4) in LDS; a code whose
 * total exceeds the LDS of one workgroup gives LDPC_ERR_UNSUPPORTED.
 */
ldpc_status ldpc_encode(ldpc_encoder_t e, const uint8_t *msg, int32_t batch, uint8_t *cw, hipStream_t stream);

/*
 * BPSK over AWGN (Sec. II-B, Eq. 4 with lambda = log P(0)/P(1)): x = 1 - 2c,
 * y = x + sigma z, lambda = 2 y / sigma^2, computed in FP64 and written as FP32
 * (flags 0) or FP64 (LDPC_LLR_F64).  cw [batch][n] bytes (nonzero = 1) in, llr
 * [batch][n] out (16-byte aligned), device memory.  The noise is counter-based
 * (Philox4x64-10 of Salmon et al., SC 2011, then Box-Muller): word w = first_word
 * + b, positions 4j..4j+3 take the block of counter (w, j, noise_stream, 0) under
 * key (seed, 2); the pair (x0, x1) gives positions 4j (cosine) and 4j+1 (sine),
 * (x2, x3) positions 4j+2 and 4j+3, with u1 = ((x0 >> 11) + 1) 2^-53 and
 * u2 = (x1 >> 11) 2^-53, z = sqrt(-2 ln u1) (cos | sin)(2 pi u2).  Any block of
 * words can be drawn on its own; noise_stream separates draws of the same words
 * (one per Eb/N0 point, say).  sigma2 must be finite and > 0.
 */
ldpc_status ldpc_channel_awgn(const uint8_t *cw, int32_t batch, int32_t n, double sigma2, uint64_t seed,
                              uint64_t noise_stream, int64_t first_word, uint32_t flags, void *llr,
                              hipStream_t stream);

/*
 * Random messages, their codewords and their channel LLRs in one launch.  The
 * message bits of word w come from key (seed, 1), counter (w, j, 0, 0): block j
 * gives bits 256 j .. 256 j + 255, bit i = bit (i mod 64) of output (i div 64)
 * mod 4; they do not depend on noise_stream, so every Eb/N0 point of a sweep sees
 * the same words.  Outputs cw [batch][n] and llr [batch][n] as in
 * ldpc_channel_awgn, and msg [batch][k] bytes if msg is not NULL.  Equal to
 * ldpc_encode of those messages followed by ldpc_channel_awgn, bit for bit.
 */
ldpc_status ldpc_generate(ldpc_encoder_t e, int32_t batch, uint64_t seed, uint64_t noise_stream, int64_t first_word,
                          double sigma2, uint32_t flags, uint8_t *msg, uint8_t *cw, void *llr, hipStream_t stream);

/*
 * Decision errors against the transmitted codewords (bit and word error counts
 * behind BER and FER): counts[0] += positions where hard != cw, counts[1] += the
 * same over message positions, counts[2] += words with any error.  hard, cw
 * [batch][n] bytes (nonzero = 1); counts: 3 device uint64, 8-byte aligned, added
 * to (the caller clears them), so several batches accumulate.
 */
ldpc_status ldpc_count_errors(ldpc_encoder_t e, const uint8_t *hard, const uint8_t *cw, int32_t batch,
                              uint64_t *counts, hipStream_t stream);

/*
 * Syndrome test of Eq. 1 (H z^T = 0 over GF(2)) on a batch of hard decisions, the
 * test the decoders apply to stop a word early: ok[b] = 1 iff every check of g has an
 * even number of ones among word b's decisions, else 0.  hard_bits: device
 * [batch][n] bytes (nonzero = 1), e.g. a decoder's hard_bits; ok: device [batch]
 * bytes, written.  Tells a word that satisfies every check at the iteration limit
 * (iters_used = max_iters) from one that does not.  batch = 0 is a no-op.
 */
ldpc_status ldpc_syndrome(ldpc_graph_t g, const uint8_t *hard_bits, int32_t batch, uint8_t *ok, hipStream_t stream);

const char *ldpc_status_string(ldpc_status s);
const char *ldpc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LDPC_H */
