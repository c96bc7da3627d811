"""Seeded parity-check matrix constructions.

The paper (Sec. II, Eq. 1) defines a binary LDPC code by an m x n parity-check
matrix H with n_c ones per column and n_v ones per row, and its experiments
(Sec. IV) use Gallager-type regular matrices whose construction it only cites.
This module builds the matrices the workloads need:

* ``gallager_band``  -- Gallager's permuted-band construction (needs dc | n);
* ``socket_regular`` -- exact (dv, dc)-regular random matrix by socket matching,
  with duplicate edges and (optionally) 4-cycles repaired by degree-preserving
  endpoint swaps (used where dc does not divide n);
* ``qc_lift``        -- quasi-cyclic lifting of a random protograph by
  circulant permutation blocks (block (i, j) with shift s links row r of the
  block row to column (r + s) mod Z of the block column);
* ``fig1_matrix``    -- the 4 x 8 (2,4) example matrix of Fig. 1.

A code is returned as a ``Code`` (CSR of H, rows sorted).  Nothing here
decodes: the module holds no sum-product arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_ROOT = 220104265


def rng_for(cfg: int, purpose: int, *sub: int) -> np.random.Generator:
    """Independent numpy stream keyed by (config, purpose, sub-keys)."""
    return np.random.default_rng([SEED_ROOT, int(cfg), int(purpose), *[int(s) for s in sub]])


@dataclass
class Code:
    """Binary parity-check matrix H (m x n) stored as CSR, column indices sorted per row."""

    m: int
    n: int
    indptr: np.ndarray  # int32 [m+1]
    indices: np.ndarray  # int32 [nnz]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def dense(self) -> np.ndarray:
        h = np.zeros((self.m, self.n), dtype=np.uint8)
        rows = np.repeat(np.arange(self.m), np.diff(self.indptr))
        h[rows, self.indices] = 1
        return h

    def row_degrees(self) -> np.ndarray:
        return np.diff(self.indptr).astype(np.int64)

    def col_degrees(self) -> np.ndarray:
        return np.bincount(self.indices, minlength=self.n).astype(np.int64)

    def csc(self):
        """(indptr over columns, row indices) of the same matrix, rows ascending per column."""
        rows = np.repeat(np.arange(self.m, dtype=np.int64), np.diff(self.indptr))
        order = np.lexsort((rows, self.indices))
        cptr = np.zeros(self.n + 1, dtype=np.int64)
        np.cumsum(np.bincount(self.indices, minlength=self.n), out=cptr[1:])
        return cptr.astype(np.int32), rows[order].astype(np.int32)


def from_edges(m: int, n: int, chk: np.ndarray, var: np.ndarray, name: str = "", meta=None) -> Code:
    chk = np.asarray(chk, dtype=np.int64)
    var = np.asarray(var, dtype=np.int64)
    order = np.lexsort((var, chk))
    chk, var = chk[order], var[order]
    key = chk * n + var
    if key.size and np.any(key[1:] == key[:-1]):
        raise ValueError("duplicate edge in parity-check matrix")
    indptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(chk, minlength=m), out=indptr[1:])
    return Code(m, n, indptr.astype(np.int32), var.astype(np.int32), name, dict(meta or {}))


def from_dense(h: np.ndarray, name: str = "") -> Code:
    h = np.asarray(h)
    c, v = np.nonzero(h)
    return from_edges(h.shape[0], h.shape[1], c, v, name)


def fig1_matrix() -> Code:
    """The (2,4) n=8 parity-check matrix printed in Fig. 1."""
    h = np.array(
        [
            [1, 1, 0, 0, 0, 1, 1, 0],
            [0, 0, 1, 1, 1, 0, 0, 1],
            [1, 1, 0, 0, 0, 1, 0, 1],
            [0, 0, 1, 1, 1, 0, 1, 0],
        ],
        dtype=np.uint8,
    )
    return from_dense(h, "fig1")


def gallager_band(n: int, dv: int, dc: int, rng: np.random.Generator, name: str = "") -> Code:
    """Gallager's permuted-band construction.

    Band 0 has n/dc rows, row i covering columns [i*dc, (i+1)*dc).  Band b
    (b = 1..dv-1) is band 0 with its columns permuted by a seeded permutation.
    Every band partitions the columns, so each column has weight dv and every
    row weight dc.
    """
    if n % dc:
        raise ValueError("permuted-band construction needs dc | n")
    rows_per_band = n // dc
    chk, var = [], []
    base = np.arange(n)
    for b in range(dv):
        perm = base if b == 0 else rng.permutation(n)
        chk.append(b * rows_per_band + base // dc)
        var.append(perm)
    m = rows_per_band * dv
    return from_edges(m, n, np.concatenate(chk), np.concatenate(var), name or f"band({dv},{dc})n{n}",
                      {"construction": "gallager_band", "dv": dv, "dc": dc})


def _four_cycle_pairs(m: int, n: int, chk: np.ndarray, var: np.ndarray):
    """Check pairs (c1 < c2) that share two or more variables."""
    import scipy.sparse as sp

    h = sp.csr_matrix((np.ones(chk.size, dtype=np.int32), (chk, var)), shape=(m, n))
    h.data[:] = 1
    a = (h @ h.T).tocoo()
    sel = (a.row < a.col) & (a.data >= 2)
    return a.row[sel], a.col[sel]


def socket_regular(n: int, dv: int, dc: int, rng: np.random.Generator, girth6: bool = True,
                   name: str = "", max_rounds: int = 20000) -> Code:
    """Exact (dv, dc)-regular random H by socket matching plus repair swaps.

    Each variable owns dv sockets and each check dc sockets; a seeded random
    permutation matches them.  Duplicate edges, and 4-cycles when ``girth6``,
    are repaired by swapping the check endpoints of an offending edge and a
    randomly chosen edge, which keeps every degree exact.
    """
    if (n * dv) % dc:
        raise ValueError("n*dv must be a multiple of dc")
    m = n * dv // dc
    var = np.repeat(np.arange(n, dtype=np.int64), dv)
    chk = rng.permutation(np.repeat(np.arange(m, dtype=np.int64), dc))
    nE = var.size
    for _ in range(max_rounds):
        key = chk * n + var
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = order[1:][ks[1:] == ks[:-1]]
        bad = list(dup)
        if not bad and girth6:
            c1, c2 = _four_cycle_pairs(m, n, chk, var)
            if c1.size:
                # one offending edge per check pair: (c1, a shared variable)
                pos = {}
                for e in range(nE):
                    pos.setdefault((int(chk[e]), int(var[e])), e)
                vars_of = {}
                for e in range(nE):
                    vars_of.setdefault(int(chk[e]), set()).add(int(var[e]))
                for a, b in zip(c1.tolist(), c2.tolist()):
                    shared = sorted(vars_of[a] & vars_of[b])
                    bad.append(pos[(a, shared[0])])
        if not bad:
            return from_edges(m, n, chk, var, name or f"socket({dv},{dc})n{n}",
                              {"construction": "socket", "dv": dv, "dc": dc, "girth6": girth6})
        for e in bad:
            e2 = int(rng.integers(nE))
            chk[e], chk[e2] = chk[e2], chk[e]
    raise RuntimeError("socket construction did not converge")


def qc_protograph(rows: int, cols: int, Z: int, rng: np.random.Generator,
                  col_w=(3, 10)) -> np.ndarray:
    """Random base matrix: -1 = zero block, s in [0, Z) = circulant shift.

    Column j gets weight uniform in [col_w[0], col_w[1]] on distinct rows; a
    base with a row of weight < 2 is redrawn.
    """
    while True:
        base = -np.ones((rows, cols), dtype=np.int64)
        for j in range(cols):
            w = int(rng.integers(col_w[0], col_w[1] + 1))
            rr = rng.choice(rows, size=w, replace=False)
            base[rr, j] = rng.integers(0, Z, size=w)
        if np.all((base >= 0).sum(axis=1) >= 2):
            return base


def qc_lift(base: np.ndarray, Z: int, name: str = "") -> Code:
    """Lift a base matrix by Z x Z circulant permutations (row r -> column (r+s) mod Z)."""
    rows, cols = base.shape
    chk, var = [], []
    r = np.arange(Z, dtype=np.int64)
    for i in range(rows):
        for j in range(cols):
            s = int(base[i, j])
            if s < 0:
                continue
            chk.append(i * Z + r)
            var.append(j * Z + (r + s) % Z)
    return from_edges(rows * Z, cols * Z, np.concatenate(chk), np.concatenate(var),
                      name or f"qc{rows}x{cols}Z{Z}", {"construction": "qc", "Z": Z, "base": base.tolist()})


def tree_code(n_target: int, rng: np.random.Generator, max_deg: int = 4) -> Code:
    """Random cycle-free Tanner graph: each new check joins one existing variable and new leaves."""
    nv = 1
    chk, var = [], []
    c = 0
    while True:
        d = int(rng.integers(2, max_deg + 1))
        if nv + d - 1 > n_target:
            d = n_target - nv + 1
            if d < 2:
                break
        anchor = int(rng.integers(nv))
        members = [anchor] + list(range(nv, nv + d - 1))
        nv += d - 1
        chk += [c] * d
        var += members
        c += 1
        if nv >= n_target:
            break
    pv = rng.permutation(nv)
    pc = rng.permutation(c)
    return from_edges(c, nv, pc[np.array(chk)], pv[np.array(var)], f"tree{nv}")


def girth_at_least_6(code: Code) -> bool:
    rows = np.repeat(np.arange(code.m), np.diff(code.indptr))
    c1, _ = _four_cycle_pairs(code.m, code.n, rows, code.indices.astype(np.int64))
    return c1.size == 0
