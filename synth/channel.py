"""BPSK over AWGN and the channel LLR (Eq. 4; Sec. III-B).

Sign convention: bit c maps to x = 1 - 2c (0 -> +1, 1 -> -1), and the channel
LLR is lambda = log P(c=0|y) / P(c=1|y) = 2 y / sigma^2.  The paper prints the
ratio the other way round with the mirrored mapping; the two conventions differ
by one global sign, and this one makes the check rule of Eq. 5 valid for odd
check degrees as well.

sigma^2 = 1 / (2 R 10^(Eb/N0 / 10)) with R = k/n the true code rate (Eb is
energy per information bit).
"""
from __future__ import annotations

import numpy as np


def sigma2(ebn0_db: float, rate: float) -> float:
    return 1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))


def bpsk(cw: np.ndarray) -> np.ndarray:
    return 1.0 - 2.0 * np.asarray(cw, dtype=np.float64)


def awgn_llr(cw: np.ndarray, s2: float, rng: np.random.Generator) -> np.ndarray:
    """FP64 LLRs 2y/sigma^2 with y = (1 - 2c) + sigma * N(0, 1)."""
    x = bpsk(cw)
    y = x + np.sqrt(s2) * rng.standard_normal(x.shape)
    return 2.0 * y / s2


def noiseless_llr(cw: np.ndarray, s2: float) -> np.ndarray:
    return 2.0 * bpsk(cw) / s2
