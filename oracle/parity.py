"""ORACLE -- test infrastructure only.

Parity rule between the FP32 GPU decoder and the FP64 oracle.

Per word:
  * hard decisions and iterations used are identical (P-hard).  A word whose
    decisions differ only on bits with |L| < 1e-3 in either implementation is an
    allowed tie exception and is counted.
  * posteriors (P-post): |L_gpu - L_oracle| <= 1e-4 * max(|L_oracle|, 1) for every
    bit, unless the word is ill-conditioned.  Loopy sum-product amplifies any
    rounding along a long decoding trajectory; the FP64 oracle itself moves by
    ~1e-4..1e-3 on such words when its inputs are perturbed by one FP32 ulp.
    For a word above 1e-4 the oracle is re-run on the same LLRs perturbed by a
    random +-1 FP32 ulp per bit (``TRIALS`` times); the word passes if the GPU
    error is at most ``FACTOR`` times the largest deviation the oracle shows under
    those perturbations (with identical iteration counts).  Only oracle runs enter
    this bound, never GPU output.
"""
from __future__ import annotations

import numpy as np

TIE = 1e-3
REL = 1e-4
TRIALS = 6
FACTOR = 4.0


def _rel(a, b):
    return np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64)) / np.maximum(np.abs(b), 1.0)


def oracle_sensitivity(oracle, code, llr_row, T, early_stop, ref_post, ref_iters, trials=TRIALS, seed=0):
    """Largest relative posterior change of the FP64 oracle under +-1 FP32-ulp input perturbations."""
    rng = np.random.default_rng(seed)
    x = np.asarray(llr_row, dtype=np.float64)
    ulp = np.spacing(np.abs(x).astype(np.float32)).astype(np.float64)
    xs = np.stack([x + rng.choice([-1.0, 1.0], size=x.shape) * ulp for _ in range(trials)])
    _, pp, ip, _ = oracle.decode(code, xs, T, early_stop)
    worst = 0.0
    for k in range(trials):
        if ip[k] != ref_iters:
            return np.inf  # the trajectory itself is unstable at this word
        worst = max(worst, float(_rel(pp[k], ref_post).max()))
    return worst


def compare(o_hard, o_post, o_iters, g_hard, g_post, g_iters, oracle=None, code=None, llr=None, T=None,
            early_stop=True):
    o_hard, g_hard = np.asarray(o_hard), np.asarray(g_hard)
    o_post, g_post = np.asarray(o_post, dtype=np.float64), np.asarray(g_post, dtype=np.float64)
    o_iters, g_iters = np.asarray(o_iters), np.asarray(g_iters)
    B = o_hard.shape[0]
    diff_bits = o_hard != g_hard
    word_diff = diff_bits.any(axis=1) | (o_iters != g_iters)
    tie_bits = (np.abs(o_post) < TIE) | (np.abs(g_post) < TIE)
    tie_ok = ~np.any(diff_bits & ~tie_bits, axis=1) & np.any(tie_bits, axis=1)
    bad_words = word_diff & ~tie_ok
    per_word = _rel(g_post, o_post).max(axis=1) if B else np.zeros(0)
    over = np.flatnonzero((per_word > REL) & ~word_diff)
    conditioned, unexplained = [], []
    for b in over:
        if oracle is None:
            unexplained.append(int(b))
            continue
        s = oracle_sensitivity(oracle, code, llr[b], T, early_stop, o_post[b], o_iters[b], seed=int(b))
        (conditioned if per_word[b] <= FACTOR * s else unexplained).append(int(b))
    return dict(
        words=B,
        mismatched_words=int(bad_words.sum()),
        tie_exceptions=int((word_diff & tie_ok).sum()),
        post_max_rel=float(per_word.max()) if B else 0.0,
        post_p99_rel=float(np.percentile(per_word, 99)) if B else 0.0,
        words_over_1e4=int(len(over)),
        ill_conditioned_words=conditioned,
        bad_post_words=unexplained,
    )


def assert_parity(stats, allow_tie_fraction: float = 0.01):
    assert stats["mismatched_words"] == 0, stats
    assert stats["tie_exceptions"] <= max(1, allow_tie_fraction * stats["words"]), stats
    assert not stats["bad_post_words"], stats
