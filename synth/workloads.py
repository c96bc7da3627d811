"""The synthetic workloads (codes, batch shapes, channel points), seeded.

Config numbers:
  1  (3,6) n=96 Gallager band, 1000 words, 2.0 dB, FP64 LLRs, 20 iterations
  2  (3,6) n=4096 socket code without 4-cycles, 65536 words, 1.0..3.0 dB, 50 iterations
  3  quasi-cyclic 22x44 protograph lifted by Z=256 (n=11264), 16384 words, 1.5 dB, 30 iterations
  4  mixed batch of six codes, 4096 words round-robin, per-code Eb/N0 in [1, 4] dB, 50 iterations
  5  (3,6) n=1024, unrolled 10 iterations with per-edge weights N(1, 0.1^2), 4096 words, 2.0 dB
  6  Table I: Gallager bands n=1032, d_c=12, d_v in {9, 6, 3}, 1000 words each, 3.0 dB, 10 iterations

Every random draw comes from ``codes.rng_for(cfg, purpose, ...)`` with purpose
0 = H, 1 = information bits, 2 = noise, 3 = weights, 4 = per-code Eb/N0.  Words
are generated in blocks of ``BLOCK`` so any block can be regenerated on its own.
The paper's experiments use Gallager-type regular codes with random vectors and
no dataset; these stand in for them.
"""
from __future__ import annotations

import functools
from dataclasses import dataclass

import numpy as np

from . import channel, codes, gf2

BLOCK = 1024


@functools.lru_cache(maxsize=None)
def code(name: str) -> codes.Code:
    """Named codes of the workloads (cached per process)."""
    if name == "c1":
        return codes.gallager_band(96, 3, 6, codes.rng_for(1, 0), "band(3,6)n96")
    if name == "c2":
        return codes.socket_regular(4096, 3, 6, codes.rng_for(2, 0), True, "socket(3,6)n4096")
    if name == "c3":
        base = codes.qc_protograph(22, 44, 256, codes.rng_for(3, 0))
        return codes.qc_lift(base, 256, "qc22x44Z256")
    if name == "c5":
        return codes.socket_regular(1024, 3, 6, codes.rng_for(5, 0), True, "socket(3,6)n1024")
    if name.startswith("c4_"):
        i = int(name[3:])
        r = codes.rng_for(4, 0, i)
        if i == 0:
            return codes.socket_regular(128, 3, 6, r, True, "socket(3,6)n128")
        if i == 1:
            return codes.socket_regular(16384, 3, 6, r, True, "socket(3,6)n16384")
        if i == 2:
            return codes.gallager_band(1024, 3, 4, r, "band(3,4)n1024")
        if i == 3:
            return codes.socket_regular(2048, 3, 12, r, True, "socket(3,12)n2048")
        if i == 4:
            return codes.socket_regular(4000, 3, 15, r, True, "socket(3,15)n4000")
        if i == 5:
            base = codes.qc_protograph(22, 44, 128, r)
            return codes.qc_lift(base, 128, "qc22x44Z128")
    if name == "paper_r14":
        return codes.gallager_band(1032, 9, 12, codes.rng_for(6, 0, 0), "band(9,12)n1032")
    if name == "paper_r12":
        return codes.gallager_band(1032, 6, 12, codes.rng_for(6, 0, 1), "band(6,12)n1032")
    if name == "paper_r34":
        return codes.gallager_band(1032, 3, 12, codes.rng_for(6, 0, 2), "band(3,12)n1032")
    raise KeyError(name)


@functools.lru_cache(maxsize=None)
def systematic(name: str) -> gf2.Systematic:
    return gf2.systematic(code(name))


def rate(name: str) -> float:
    s = systematic(name)
    return s.k / s.n


@dataclass
class Words:
    cw: np.ndarray  # uint8 [B, n] transmitted codewords
    llr: np.ndarray  # [B, n] channel LLRs (float64 or float32)
    sigma2: float


def words(name: str, cfg: int, snr_key: int, ebn0_db: float, start: int, count: int,
          fp32: bool = True, code_key: int = 0) -> Words:
    """Codewords [start, start+count) of a code's stream and their LLRs at Eb/N0.

    Information bits depend on (cfg, code_key, block) only, so every Eb/N0 point
    sees the same transmitted words; the noise depends on (cfg, code_key, snr_key, block).
    FP32 workloads round the FP64 LLRs to FP32 once.
    """
    s = systematic(name)
    s2 = channel.sigma2(ebn0_db, s.k / s.n)
    b0, b1 = start // BLOCK, (start + count + BLOCK - 1) // BLOCK
    cws, llrs = [], []
    for blk in range(b0, b1):
        msg = codes.rng_for(cfg, 1, code_key, blk).integers(0, 2, size=(BLOCK, s.k), dtype=np.uint8)
        cw = s.encode(msg)
        llr = channel.awgn_llr(cw, s2, codes.rng_for(cfg, 2, code_key, snr_key, blk))
        cws.append(cw)
        llrs.append(llr.astype(np.float32) if fp32 else llr)
    cw = np.concatenate(cws)
    llr = np.concatenate(llrs)
    lo = start - b0 * BLOCK
    return Words(np.ascontiguousarray(cw[lo:lo + count]), np.ascontiguousarray(llr[lo:lo + count]), s2)


# ---- workload descriptions -------------------------------------------------

C1 = dict(code="c1", batch=1000, ebn0=2.0, max_iters=20, fp32=False, cfg=1)
C2 = dict(code="c2", batch=65536, ebn0s=(1.0, 1.5, 2.0, 2.5, 3.0), max_iters=50, fp32=True, cfg=2)
C3 = dict(code="c3", batch=16384, ebn0=1.5, max_iters=30, fp32=True, cfg=3)
C4_CODES = tuple(f"c4_{i}" for i in range(6))
C4 = dict(codes=C4_CODES, batch=4096, max_iters=50, fp32=True, cfg=4)
C5 = dict(code="c5", batch=4096, ebn0=2.0, iters=10, fp32=True, cfg=5)
# Table I of the paper: n = 1032, 12 ones per row, 9 / 6 / 3 per column (design rates 1/4, 1/2,
# 3/4), 10 decoding iterations (a preset count, no early stop), 1000 vectors.  The paper gives no
# channel point; at 3.0 dB the rate-1/2 and 3/4 codes decode some words and not others.
PAPER = dict(codes=("paper_r14", "paper_r12", "paper_r34"), batch=1000, iters=10, ebn0=3.0, fp32=True, cfg=6)


def c4_ebn0() -> np.ndarray:
    """Per-code Eb/N0 of the mixed batch: uniform on the 0.1 dB grid in [1, 4]."""
    return codes.rng_for(4, 4).integers(10, 41, size=len(C4_CODES)) / 10.0


def c4_counts(batch: int = 4096) -> list[int]:
    """Word i of the mixed batch goes to code i mod 6."""
    q = len(C4_CODES)
    return [batch // q + (1 if i < batch % q else 0) for i in range(q)]


def c5_weights(T: int = 10) -> np.ndarray:
    E = code("c5").nnz
    return codes.rng_for(5, 3).normal(1.0, 0.1, size=(T, E)).astype(np.float32)


def paper_words(i: int, count: int | None = None) -> Words:
    """The Table I vectors of code i (0: rate 1/4, 1: 1/2, 2: 3/4)."""
    return words(PAPER["codes"][i], PAPER["cfg"], 0, PAPER["ebn0"], 0, count or PAPER["batch"],
                 fp32=PAPER["fp32"], code_key=i)
