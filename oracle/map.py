"""ORACLE -- test infrastructure only.

Exact bitwise MAP by enumerating the codebook.  With lambda_i = log P(y_i|0)/P(y_i|1),
log P(y | c) = const + sum_i (1 - 2 c_i) lambda_i / 2, so the bitwise posterior LLR is

    L_v = logsumexp_{c: c_v = 0} s(c) - logsumexp_{c: c_v = 1} s(c),  s(c) = sum_i (1 - 2 c_i) lambda_i / 2.

Sum-product decoding computes exactly this on a cycle-free Tanner graph once the
messages have crossed the graph (Sec. II-B cites the standard derivations); this
enumeration is the ground truth it is compared with.  Feasible for k <= ~18.
"""
from __future__ import annotations

import numpy as np
from scipy.special import logsumexp


def codebook(G: np.ndarray) -> np.ndarray:
    """Every codeword m G (mod 2) of a k x n generator G."""
    G = np.asarray(G, dtype=np.int64)
    k = G.shape[0]
    msgs = (np.arange(1 << k, dtype=np.int64)[:, None] >> np.arange(k, dtype=np.int64)[None, :]) & 1
    return ((msgs @ G) & 1).astype(np.uint8)


def bitwise_map(G: np.ndarray, llr: np.ndarray) -> np.ndarray:
    """Bitwise MAP LLRs [B, n] for channel LLRs [B, n] (FP64)."""
    cb = codebook(G).astype(np.float64)  # [2^k, n]
    llr = np.atleast_2d(np.asarray(llr, dtype=np.float64))
    s = 0.5 * llr @ (1.0 - 2.0 * cb).T  # [B, 2^k]
    out = np.empty_like(llr)
    for v in range(llr.shape[1]):
        zero = cb[:, v] == 0
        out[:, v] = logsumexp(s[:, zero], axis=1) - logsumexp(s[:, ~zero], axis=1)
    return out
