"""Tanner-graph handle (ldpc_graph_create / ldpc_graph_destroy)."""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import check, lib

CSR, CSC = 0, 1


class Graph:
    """Immutable device-resident Tanner graph of a parity-check matrix H (m x n)."""

    def __init__(self, m: int, n: int, ptr, idx, fmt: int = CSR):
        ptr = np.ascontiguousarray(ptr, dtype=np.int32)
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        h = ctypes.c_void_p()
        check("ldpc_graph_create",
              lib().ldpc_graph_create(int(m), int(n), int(fmt), ptr.ctypes.data_as(ctypes.c_void_p),
                                      idx.ctypes.data_as(ctypes.c_void_p), int(ptr[-1]) if ptr.size else 0,
                                      ctypes.byref(h)))
        self._h = h
        mm, nn, dc, dv = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        ee = ctypes.c_int64()
        check("ldpc_graph_info", lib().ldpc_graph_info(h, ctypes.byref(mm), ctypes.byref(nn), ctypes.byref(ee),
                                                        ctypes.byref(dc), ctypes.byref(dv)))
        self.m, self.n, self.edges = mm.value, nn.value, ee.value
        self.max_check_deg, self.max_var_deg = dc.value, dv.value

    @classmethod
    def from_csr(cls, m, n, indptr, indices) -> "Graph":
        return cls(m, n, indptr, indices, CSR)

    @classmethod
    def from_csc(cls, m, n, indptr, indices) -> "Graph":
        return cls(m, n, indptr, indices, CSC)

    @classmethod
    def from_code(cls, code) -> "Graph":
        """From any object with m, n, indptr, indices (CSR of H)."""
        return cls(code.m, code.n, code.indptr, code.indices, CSR)

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def edge_arrays(self):
        """(check_of_edge, var_of_edge) int32 arrays in the library's edge numbering (CSR order)."""
        c = np.zeros(self.edges, dtype=np.int32)
        v = np.zeros(self.edges, dtype=np.int32)
        check("ldpc_graph_edges", lib().ldpc_graph_edges(self._h, c.ctypes.data_as(ctypes.c_void_p),
                                                          v.ctypes.data_as(ctypes.c_void_p)))
        return c, v

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ldpc_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):  # pragma: no cover - interpreter shutdown order
        try:
            self.close()
        except Exception:
            pass
