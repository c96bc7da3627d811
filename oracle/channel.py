"""ORACLE -- test infrastructure only.

The random draws of on-device word generation, written from their definitions:

* Philox4x64-10, the counter-based generator of Salmon, Moraes, Dror and Shaw,
  "Parallel random numbers: as easy as 1, 2, 3" (SC 2011): a 256-bit counter
  (four 64-bit words) and a 128-bit key; each of 10 rounds multiplies counter
  words 0 and 2 by fixed 64-bit constants, splits the 128-bit products into
  high and low halves, and rearranges them with XORs of the other two words and
  the key; the key is bumped by two Weyl constants between rounds.
* Message bits of word w: key (seed, 1); block j = philox(counter (w, j, 0, 0))
  gives bits 256 j .. 256 j + 255, bit i = bit (i mod 64) of output (i div 64) mod 4.
* Noise of word w at variable v: key (seed, 2); block philox(counter (w, v div 4,
  stream, 0)) = (x0, x1, x2, x3) feeds two Box-Muller pairs:
  u1 = (x0 >> 11 + 1) 2^-53 in (0, 1], u2 = (x1 >> 11) 2^-53 in [0, 1),
  r = sqrt(-2 ln u1), z(4j) = r cos(2 pi u2), z(4j+1) = r sin(2 pi u2); (x2, x3)
  give z(4j+2), z(4j+3) the same way.
* Channel (Sec. II-B, Eq. 4 with lambda = log P(0)/P(1)): BPSK x = 1 - 2c,
  y = x + sigma z, lambda = 2 y / sigma^2, in FP64; FP32 outputs round it once.

numpy only, FP64, vectorised over words but otherwise step by step.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

DOMAIN_MESSAGE = 1
DOMAIN_NOISE = 2


def mulhilo(a: np.ndarray, b: np.uint64):
    """(high, low) 64-bit halves of the 128-bit product a * b, from four 32 x 32-bit products."""
    a = np.asarray(a, dtype=np.uint64)
    a0, a1 = a & _LO32, a >> _S32
    b0, b1 = b & _LO32, b >> _S32
    with np.errstate(over="ignore"):
        p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
        mid = (p00 >> _S32) + (p01 & _LO32) + (p10 & _LO32)
        hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
        lo = a * b
    return hi, lo


def philox4x64(ctr: np.ndarray, key) -> np.ndarray:
    """Philox4x64-10 of counters [N, 4] (uint64) under key (k0, k1): outputs [N, 4] uint64."""
    c = np.array(ctr, dtype=np.uint64).reshape(-1, 4)
    r0, r1, r2, r3 = (c[:, i].copy() for i in range(4))
    k0, k1 = np.uint64(key[0]), np.uint64(key[1])
    for _ in range(10):
        hi0, lo0 = mulhilo(r0, M0)
        hi1, lo1 = mulhilo(r2, M1)
        r0, r1, r2, r3 = hi1 ^ r1 ^ k0, lo1, hi0 ^ r3 ^ k1, lo0
        with np.errstate(over="ignore"):
            k0, k1 = k0 + W0, k1 + W1
    return np.stack([r0, r1, r2, r3], axis=1)


def messages(seed: int, first_word: int, batch: int, k: int) -> np.ndarray:
    """Message bits [batch, k] (uint8) of words first_word .. first_word + batch - 1."""
    nblk = (k + 255) // 256
    out = np.zeros((batch, nblk * 256), dtype=np.uint8)
    for j in range(nblk):
        ctr = np.zeros((batch, 4), dtype=np.uint64)
        ctr[:, 0] = np.arange(first_word, first_word + batch, dtype=np.uint64)
        ctr[:, 1] = j
        x = philox4x64(ctr, (seed, DOMAIN_MESSAGE))  # [batch, 4]
        for q in range(4):
            bits = (x[:, q:q + 1] >> np.arange(64, dtype=np.uint64)[None, :]) & np.uint64(1)
            out[:, 256 * j + 64 * q:256 * j + 64 * q + 64] = bits.astype(np.uint8)
    return out[:, :k]


def box_muller(xa: np.ndarray, xb: np.ndarray):
    """Two standard normals from two 64-bit words each (the reading above)."""
    u1 = ((xa >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * 2.0 ** -53
    u2 = (xb >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(u1))
    t = (2.0 * np.pi) * u2
    return r * np.cos(t), r * np.sin(t)


def normals(seed: int, stream: int, first_word: int, batch: int, n: int) -> np.ndarray:
    """Standard normal draws [batch, n] (FP64) of words first_word .. first_word + batch - 1."""
    nblk = (n + 3) // 4
    z = np.zeros((batch, nblk * 4), dtype=np.float64)
    for j in range(nblk):
        ctr = np.zeros((batch, 4), dtype=np.uint64)
        ctr[:, 0] = np.arange(first_word, first_word + batch, dtype=np.uint64)
        ctr[:, 1] = j
        ctr[:, 2] = stream
        x = philox4x64(ctr, (seed, DOMAIN_NOISE))
        z[:, 4 * j], z[:, 4 * j + 1] = box_muller(x[:, 0], x[:, 1])
        z[:, 4 * j + 2], z[:, 4 * j + 3] = box_muller(x[:, 2], x[:, 3])
    return z[:, :n]


def awgn_llr(cw: np.ndarray, sigma2: float, seed: int, stream: int = 0, first_word: int = 0,
             f64: bool = False) -> np.ndarray:
    """Channel LLRs of codewords cw [B, n] (Eq. 4): 2 (1 - 2c + sigma z) / sigma^2."""
    cw = np.atleast_2d(np.asarray(cw, dtype=np.uint8))
    B, n = cw.shape
    z = normals(seed, stream, first_word, B, n)
    sigma = np.sqrt(sigma2)
    x = 1.0 - 2.0 * cw.astype(np.float64)
    y = x + sigma * z
    lam = 2.0 * y / sigma2
    return lam if f64 else lam.astype(np.float32)


def error_counts(hard: np.ndarray, cw: np.ndarray, info: np.ndarray) -> np.ndarray:
    """[coded bit errors, message bit errors, word errors] of decisions against codewords."""
    diff = np.atleast_2d(np.asarray(hard, dtype=np.uint8)) != np.atleast_2d(np.asarray(cw, dtype=np.uint8))
    return np.array([diff.sum(), diff[:, np.asarray(info)].sum(), diff.any(axis=1).sum()], dtype=np.int64)
