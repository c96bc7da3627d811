"""ORACLE -- test infrastructure only.

Parity rule between the FP32 GPU decoder and the FP64 oracle.

Per word (every rule below uses oracle runs only to decide what is excused):

* decisions and iterations (P-hard).  Hard decisions and iterations used are
  identical.  Two exceptions, both ties of Eq. 8 at L = 0, counted and reported:
    - same iteration count, and every bit whose decision differs has |L| < TIE in
      the oracle or on the GPU;
    - different iteration counts t_o != t_g: the syndrome test of Eq. 1 came out
      differently at iteration t* = min(t_o, t_g).  Excused only if the oracle's own
      posterior at t* (a run of exactly t* iterations) has a bit with |L| < TIE, a
      decision that rounding can flip.

* posteriors (P-post).  |L_gpu - L_64| <= REL * max(|L_64|, 1) on every bit.  A word
  above that passes only if it is ill-conditioned for FP32 storage itself, which the
  FP32-storage build of the oracle decides (the same source with every stored value
  rounded to FP32, all arithmetic in FP64: what any FP32 decoder would return if each
  of its stored values were correctly rounded).  That build is run on the word's LLRs
  and on TRIALS copies perturbed by a random +-1 FP32 ulp per LLR; s32 is the largest
  relative deviation from the FP64 posterior over the runs that take the oracle's
  iteration count (if none does, the word is not excused).  The word passes iff
  s32 > REL / FACTOR (correct FP32 rounding alone already moves it to within FACTOR of
  the bound) and the GPU error is at most FACTOR * s32.

  FACTOR = 4: loopy sum-product amplifies the rounding injected at each step, so an
  FP32 decoder whose per-step error is k times that of correct rounding ends, in
  distribution, about k times further out on an ill-conditioned trajectory.  The
  one-step tests measure k (rms of the GPU's c->v error over that of correct rounding)
  at 2 to 2.5 where messages are moderate (C1, C2 at 1.0 dB, C4's low-SNR codes) and up
  to 5 where most messages are large (after convergence, where the hardware log2's
  error of about one ulp of log2(s/d) dominates and no trajectory is ill-conditioned);
  on every FP32-ill-conditioned word seen so far the GPU error has stayed within twice
  the largest of the 1 + TRIALS = 9 FP32-storage deviations (worst_conditioned_ratio),
  so FACTOR = 4 keeps a factor-2 margin without admitting an error that correct FP32
  rounding could not produce on that word.
"""
from __future__ import annotations

import numpy as np

TIE = 1e-3
REL = 1e-4
TRIALS = 8
FACTOR = 4.0


def _rel(a, b):
    return np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64)) / np.maximum(np.abs(b), 1.0)


def fp32_sensitivity(oracle, code, llr_row, T, early_stop, ref_post, ref_iters, trials=TRIALS, seed=0):
    """Largest relative deviation from the FP64 posterior of the FP32-storage oracle on this
    word's LLRs and on `trials` copies perturbed by +-1 FP32 ulp per LLR, over the runs
    whose iteration count equals ref_iters (0.0 and runs = 0 if none does)."""
    rng = np.random.default_rng(seed)
    x = np.asarray(llr_row, dtype=np.float64)
    ulp = np.spacing(np.abs(x).astype(np.float32)).astype(np.float64)
    xs = np.stack([x] + [x + rng.choice([-1.0, 1.0], size=x.shape) * ulp for _ in range(trials)])
    _, pp, ip, _, _ = oracle.decode_ex(code, xs, T, early_stop, store32=True)
    ok = ip == ref_iters
    if not ok.any():
        return 0.0, 0
    return float(max(_rel(pp[k], ref_post).max() for k in np.flatnonzero(ok))), int(ok.sum())


def compare(o_hard, o_post, o_iters, g_hard, g_post, g_iters, oracle=None, code=None, llr=None, T=None,
            early_stop=True):
    """Statistics of the GPU outputs against the oracle's under the rule above.

    oracle/code/llr/T are needed to judge the exceptions (iteration-count ties and
    FP32-ill-conditioned words); without them no exception is granted."""
    o_hard, g_hard = np.asarray(o_hard), np.asarray(g_hard)
    o_post, g_post = np.asarray(o_post, dtype=np.float64), np.asarray(g_post, dtype=np.float64)
    o_iters, g_iters = np.asarray(o_iters), np.asarray(g_iters)
    B = o_hard.shape[0]
    diff_bits = o_hard != g_hard
    tie_bits = (np.abs(o_post) < TIE) | (np.abs(g_post) < TIE)
    same_it = o_iters == g_iters
    # same iteration count: every differing decision must itself be a tie
    hard_ok = ~np.any(diff_bits & ~tie_bits, axis=1)
    tie_words = same_it & hard_ok & diff_bits.any(axis=1)
    bad = same_it & ~hard_ok
    # different iteration counts: a tie in the oracle's posterior at the deciding iteration
    for b in np.flatnonzero(~same_it):
        t_star = int(min(o_iters[b], g_iters[b]))
        excused = False
        if oracle is not None:
            _, p_t, _, _ = oracle.decode(code, np.asarray(llr[b])[None, :], t_star, False)
            excused = bool(np.any(np.abs(p_t) < TIE))
        if excused:
            tie_words[b] = True
        else:
            bad[b] = True
    per_word = _rel(g_post, o_post).max(axis=1) if B else np.zeros(0)
    exact_words = same_it & ~diff_bits.any(axis=1)
    over = np.flatnonzero((per_word > REL) & exact_words)
    conditioned, unexplained, s32s, ratios = [], [], {}, []
    for b in over:
        if oracle is None:
            unexplained.append(int(b))
            continue
        s32, runs = fp32_sensitivity(oracle, code, llr[b], T, early_stop, o_post[b], o_iters[b], seed=int(b))
        s32s[int(b)] = (s32, runs)
        if runs and s32 > 0:
            ratios.append(float(per_word[b] / s32))
        if runs and s32 > REL / FACTOR and per_word[b] <= FACTOR * s32:
            conditioned.append(int(b))
        else:
            unexplained.append(int(b))
    return dict(
        words=B,
        mismatched_words=int(bad.sum()),
        tie_exceptions=int(tie_words.sum()),
        post_max_rel=float(per_word.max()) if B else 0.0,
        post_p99_rel=float(np.percentile(per_word, 99)) if B else 0.0,
        post_median_rel=float(np.median(per_word)) if B else 0.0,
        words_over_1e4=int(len(over)),
        ill_conditioned_words=conditioned,
        fp32_sensitivity={k: round(v[0], 8) for k, v in s32s.items()},
        worst_conditioned_ratio=round(max(ratios), 3) if ratios else None,
        bad_post_words=unexplained,
    )


def assert_parity(stats, allow_tie_fraction: float = 0.01):
    assert stats["mismatched_words"] == 0, stats
    assert stats["tie_exceptions"] <= max(1, allow_tie_fraction * stats["words"]), stats
    assert not stats["bad_post_words"], stats
