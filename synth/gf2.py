"""GF(2) systematic encoder (Sec. II-A, Eqs. 2-3; Sec. III-B, systematic [I_k : P] form).

Codewords are the null space of H (Eq. 1).  Gauss-Jordan elimination of H over
GF(2) (bit-packed rows) finds one pivot per independent row; pivot columns are
scanned from n-1 down to 0 so parity positions sit at the right end where the
matrix allows.  rank = #pivots, k = n - rank.  The non-pivot columns, in
ascending order, carry the information bits; reduced row r then fixes the bit
in its pivot column as the GF(2) sum of the information bits it touches.

This is input generation: it produces the transmitted words, it never decodes.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .codes import Code


@dataclass
class Systematic:
    n: int
    rank: int
    k: int
    pivots: np.ndarray  # int64 [rank]: pivot column of reduced row r
    info: np.ndarray  # int64 [k]: information positions, ascending
    A: np.ndarray  # uint8 [rank, k]: parity(pivots[r]) = sum_j A[r, j] * m_j  (mod 2)

    def generator(self) -> np.ndarray:
        """Explicit k x n generator G with H G^T = 0 and G[:, info] = I_k."""
        g = np.zeros((self.k, self.n), dtype=np.uint8)
        g[np.arange(self.k), self.info] = 1
        g[:, self.pivots] = self.A.T
        return g

    def encode(self, msg: np.ndarray) -> np.ndarray:
        """Codewords [B, n] (uint8) from information bits [B, k] (Eq. 3, systematic)."""
        msg = np.asarray(msg, dtype=np.uint8)
        B = msg.shape[0]
        cw = np.zeros((B, self.n), dtype=np.uint8)
        cw[:, self.info] = msg
        if self.rank:
            # exact: integer sums <= k < 2^24 in float32
            par = msg.astype(np.float32) @ self.A.T.astype(np.float32)
            cw[:, self.pivots] = (par.astype(np.int64) & 1).astype(np.uint8)
        return cw


def _pack_rows(code: Code) -> np.ndarray:
    W = (code.n + 63) // 64
    rows = np.zeros((code.m, W), dtype=np.uint64)
    r = np.repeat(np.arange(code.m), np.diff(code.indptr))
    c = code.indices.astype(np.int64)
    np.bitwise_or.at(rows, (r, c >> 6), np.left_shift(np.uint64(1), (c & 63).astype(np.uint64)))
    return rows


def systematic(code: Code) -> Systematic:
    M = _pack_rows(code)
    m, n = code.m, code.n
    rank = 0
    pivots = []
    for col in range(n - 1, -1, -1):
        if rank == m:
            break
        w, b = col >> 6, np.uint64(col & 63)
        bits = (M[rank:, w] >> b) & np.uint64(1)
        hit = np.flatnonzero(bits)
        if hit.size == 0:
            continue
        p = rank + int(hit[0])
        if p != rank:
            M[[rank, p]] = M[[p, rank]]
        allbits = ((M[:, w] >> b) & np.uint64(1)).astype(bool)
        allbits[rank] = False
        if allbits.any():
            M[allbits] ^= M[rank]
        pivots.append(col)
        rank += 1
    pivots = np.array(pivots, dtype=np.int64)
    is_piv = np.zeros(n, dtype=bool)
    is_piv[pivots] = True
    info = np.flatnonzero(~is_piv).astype(np.int64)
    # unpack reduced rows restricted to info columns
    if rank:
        words = M[:rank, :]
        bits = np.unpackbits(words.view(np.uint8), axis=1, bitorder="little")[:, :n]
        A = bits[:, info].astype(np.uint8)
    else:
        A = np.zeros((0, info.size), dtype=np.uint8)
    return Systematic(n, rank, n - rank, pivots, info, A)


def gf2_rank(mat: np.ndarray) -> int:
    """Rank over GF(2) of a small dense 0/1 matrix (plain row reduction)."""
    a = (np.asarray(mat, dtype=np.uint8) & 1).copy()
    r = 0
    rows, cols = a.shape
    for c in range(cols):
        piv = np.flatnonzero(a[r:, c])
        if piv.size == 0:
            continue
        p = r + int(piv[0])
        a[[r, p]] = a[[p, r]]
        mask = a[:, c].astype(bool)
        mask[r] = False
        a[mask] ^= a[r]
        r += 1
        if r == rows:
            break
    return r

