"""Parity rule between the FP32 GPU decoder and the FP64 oracle.

Per word:
  * hard decisions and iterations used must be identical; a word whose decisions
    differ only on bits with |L| < 1e-3 (in either implementation) is an allowed
    tie exception and is counted;
  * posteriors: |L_gpu - L_oracle| <= 1e-4 * max(|L_oracle|, 1) for every bit of
    every word whose oracle iteration count is <= POST_CUT.

Loopy sum-product amplifies rounding on words that run for many iterations (two
FP64 implementations differ too), so posteriors of longer words are reported as
an error distribution instead of being asserted element-wise.
"""
from __future__ import annotations

import numpy as np

TIE = 1e-3
REL = 1e-4
POST_CUT = 20


def compare(o_hard, o_post, o_iters, g_hard, g_post, g_iters, post_cut: int = POST_CUT):
    o_hard, g_hard = np.asarray(o_hard), np.asarray(g_hard)
    o_post, g_post = np.asarray(o_post, dtype=np.float64), np.asarray(g_post, dtype=np.float64)
    o_iters, g_iters = np.asarray(o_iters), np.asarray(g_iters)
    B = o_hard.shape[0]
    diff_bits = o_hard != g_hard
    word_diff = diff_bits.any(axis=1) | (o_iters != g_iters)
    tie_bits = (np.abs(o_post) < TIE) | (np.abs(g_post) < TIE)
    # a word may differ only where a decision is a near tie
    tie_ok = ~np.any(diff_bits & ~tie_bits, axis=1) & np.any(tie_bits, axis=1)
    bad_words = word_diff & ~tie_ok
    rel = np.abs(g_post - o_post) / np.maximum(np.abs(o_post), 1.0)
    per_word = rel.max(axis=1) if rel.size else np.zeros(B)
    short = o_iters <= post_cut
    stats = dict(
        words=B,
        mismatched_words=int(bad_words.sum()),
        tie_exceptions=int((word_diff & tie_ok).sum()),
        post_checked_words=int(short.sum()),
        post_max_rel_short=float(per_word[short].max()) if short.any() else 0.0,
        post_rel_long=(np.percentile(per_word[~short], [50, 99, 100]).tolist() if (~short).any() else []),
        bad_post_words=int((per_word[short] > REL).sum()),
    )
    return stats


def assert_parity(stats, allow_tie_fraction: float = 0.01):
    assert stats["mismatched_words"] == 0, stats
    assert stats["tie_exceptions"] <= max(1, allow_tie_fraction * stats["words"]), stats
    assert stats["bad_post_words"] == 0, stats
