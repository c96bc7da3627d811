"""ORACLE -- test infrastructure only.

Systematic GF(2) encoding of an LDPC code given by its parity-check matrix H.

* A codeword is a word c with H c^T = 0 over GF(2) (Eq. 1); the codewords form
  the row space of a k x n generator G, and a message m of k bits is sent as
  c = m G (Eqs. 2-3).
* A systematic generator copies the message into k of the n positions; with
  those positions gathered first it reads [I_k : P] (Sec. III-B; Fig. 2 shows
  one such G).  Which columns hold the message is a choice -- the paper allows a
  column permutation -- and the reading used here is:
    - reduce H to reduced row echelon form over GF(2), choosing pivot columns
      from the last column (n-1) towards the first, the first row (in current
      order) with a 1 in that column becoming the next pivot row;
    - rank = number of pivots, k = n - rank;
    - the non-pivot columns, ascending, carry the message bits;
    - reduced row r says: bit pivot[r] = GF(2) sum of the message bits in the
      non-pivot columns where row r has a 1.
* G is then built explicitly (k x n) and encoding is the product m G mod 2.

Plain dense 0/1 arithmetic in numpy (one byte per bit), slow but direct.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class SystematicForm:
    n: int
    rank: int
    k: int
    pivots: np.ndarray  # int64 [rank], pivot column of reduced row r
    info: np.ndarray  # int64 [k], message positions, ascending
    G: np.ndarray  # uint8 [k, n]


def dense_h(code) -> np.ndarray:
    """H as a dense m x n 0/1 matrix from any object with m, n, indptr, indices (CSR)."""
    H = np.zeros((code.m, code.n), dtype=np.uint8)
    indptr = np.asarray(code.indptr)
    for c in range(code.m):
        H[c, np.asarray(code.indices[indptr[c]:indptr[c + 1]])] = 1
    return H


def reduce_rows(H: np.ndarray):
    """Reduced row echelon form over GF(2), pivots chosen from the last column down.

    Returns (R, pivots): R[:rank] are the reduced independent rows, pivots[r] the
    column of row r's leading 1 (every other row of R is 0 in that column)."""
    R = (np.asarray(H, dtype=np.uint8) & 1).copy()
    m, n = R.shape
    pivots = []
    rank = 0
    for col in range(n - 1, -1, -1):
        if rank == m:
            break
        below = np.flatnonzero(R[rank:, col])
        if below.size == 0:
            continue
        p = rank + int(below[0])
        if p != rank:
            R[[rank, p]] = R[[p, rank]]
        others = np.flatnonzero(R[:, col])
        others = others[others != rank]
        R[others] ^= R[rank]
        pivots.append(col)
        rank += 1
    return R[:rank], np.array(pivots, dtype=np.int64)


def systematic(code_or_h) -> SystematicForm:
    """The systematic generator of the reading above."""
    H = code_or_h if isinstance(code_or_h, np.ndarray) else dense_h(code_or_h)
    n = H.shape[1]
    R, pivots = reduce_rows(H)
    rank = pivots.size
    is_pivot = np.zeros(n, dtype=bool)
    is_pivot[pivots] = True
    info = np.flatnonzero(~is_pivot).astype(np.int64)
    k = info.size
    G = np.zeros((k, n), dtype=np.uint8)
    G[np.arange(k), info] = 1
    # column pivot[r] of G: message bit j contributes iff row r has a 1 in column info[j]
    if rank:
        G[:, pivots] = R[:, info].T
    return SystematicForm(n, rank, k, pivots, info, G)


def encode(form: SystematicForm, msg: np.ndarray) -> np.ndarray:
    """Codewords [B, n] = m G mod 2 (Eq. 3) for messages [B, k] (0/1)."""
    msg = np.atleast_2d(np.asarray(msg, dtype=np.int64) & 1)
    return ((msg @ form.G.astype(np.int64)) & 1).astype(np.uint8)


def encode_with_generator(msg: np.ndarray, G: np.ndarray) -> np.ndarray:
    """m G mod 2 for an explicitly given generator (Fig. 2)."""
    msg = np.atleast_2d(np.asarray(msg, dtype=np.int64) & 1)
    return ((msg @ np.asarray(G, dtype=np.int64)) & 1).astype(np.uint8)
