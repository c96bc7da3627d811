"""Plain flooding decode (ldpc_decode): argument marshalling for torch device tensors."""
from __future__ import annotations

import ctypes

import torch

from ._lib import LLR_F64, check, lib, stream_handle
from .graph import Graph


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def workspace_size(graph: Graph, batch: int, f64: bool = False) -> int:
    out = ctypes.c_size_t()
    check("ldpc_decode_workspace_size",
          lib().ldpc_decode_workspace_size(graph.handle, int(batch), LLR_F64 if f64 else 0, ctypes.byref(out)))
    return out.value


def decode(graph: Graph, llr: torch.Tensor, max_iters: int, early_stop: bool = True, waves: int | None = None,
           workspace: torch.Tensor | None = None, out=None, stream=None):
    """Decode llr [B, n] (cuda float32 or float64).  Returns (hard u8 [B,n], posterior f32 [B,n], iters i32 [B])."""
    if not llr.is_cuda or llr.dim() != 2 or llr.shape[1] != graph.n:
        raise ValueError("llr must be a cuda tensor of shape [B, n]")
    if llr.dtype not in (torch.float32, torch.float64):
        raise ValueError("llr must be float32 or float64")
    llr = llr.contiguous()
    B = llr.shape[0]
    f64 = llr.dtype == torch.float64
    dev = llr.device
    if out is None:
        hard = torch.empty((B, graph.n), dtype=torch.uint8, device=dev)
        post = torch.empty((B, graph.n), dtype=torch.float32, device=dev)
        iters = torch.empty((B,), dtype=torch.int32, device=dev)
    else:
        hard, post, iters = out
    need = workspace_size(graph, B, f64)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty((max(need, 1),), dtype=torch.uint8, device=dev)
    flags = LLR_F64 if f64 else 0
    h = lib()
    s = ctypes.c_void_p(stream_handle(stream))
    if waves is None:
        st = h.ldpc_decode(graph.handle, _ptr(llr), B, int(max_iters), int(bool(early_stop)), flags, _ptr(hard),
                           _ptr(post), _ptr(iters), _ptr(workspace), workspace.numel(), s)
    else:
        st = h.ldpc_decode_config(graph.handle, _ptr(llr), B, int(max_iters), int(bool(early_stop)), flags,
                                  _ptr(hard), _ptr(post), _ptr(iters), _ptr(workspace), workspace.numel(),
                                  int(waves), s)
    check("ldpc_decode", st)
    return hard, post, iters


def decode_ex(graph: Graph, llr: torch.Tensor, max_iters: int, early_stop: bool = True,
              init_cv: torch.Tensor | None = None, want_final: bool = True, stream=None):
    """ldpc_decode_ex: decode from the c->v state init_cv [B, edges] (float32, CSR edge order;
    None = zeros).  Returns (hard, posterior, iters, final_cv [B, edges] or None)."""
    if not llr.is_cuda or llr.dim() != 2 or llr.shape[1] != graph.n:
        raise ValueError("llr must be a cuda tensor of shape [B, n]")
    if llr.dtype not in (torch.float32, torch.float64):
        raise ValueError("llr must be float32 or float64")
    llr = llr.contiguous()
    B = llr.shape[0]
    f64 = llr.dtype == torch.float64
    dev = llr.device
    if init_cv is not None:
        if not init_cv.is_cuda or init_cv.dtype != torch.float32 or tuple(init_cv.shape) != (B, graph.edges):
            raise ValueError("init_cv must be a cuda float32 tensor of shape [B, edges]")
        init_cv = init_cv.contiguous()
    hard = torch.empty((B, graph.n), dtype=torch.uint8, device=dev)
    post = torch.empty((B, graph.n), dtype=torch.float32, device=dev)
    iters = torch.empty((B,), dtype=torch.int32, device=dev)
    final = torch.empty((B, graph.edges), dtype=torch.float32, device=dev) if want_final else None
    need = workspace_size(graph, B, f64)
    workspace = torch.empty((max(need, 1),), dtype=torch.uint8, device=dev)
    s = ctypes.c_void_p(stream_handle(stream))
    st = lib().ldpc_decode_ex(graph.handle, _ptr(llr), B, int(max_iters), int(bool(early_stop)),
                              LLR_F64 if f64 else 0, _ptr(init_cv) if init_cv is not None else None,
                              _ptr(final) if final is not None else None, _ptr(hard), _ptr(post), _ptr(iters),
                              _ptr(workspace), workspace.numel(), s)
    check("ldpc_decode_ex", st)
    return hard, post, iters, final


def stream_supported(graph: Graph) -> bool:
    nb, ok = ctypes.c_size_t(), ctypes.c_int32()
    check("ldpc_stream_lds_bytes", lib().ldpc_stream_lds_bytes(graph.handle, ctypes.byref(nb), ctypes.byref(ok)))
    return bool(ok.value)


def stream_lds_bytes(graph: Graph) -> int:
    """LDS bytes of one word's state in the stream form."""
    nb = ctypes.c_size_t()
    check("ldpc_stream_lds_bytes", lib().ldpc_stream_lds_bytes(graph.handle, ctypes.byref(nb), None))
    return int(nb.value)


def decode_stream(graph: Graph, llr: torch.Tensor, max_iters: int, early_stop: bool = True, threads: int = 0,
                  workspace: torch.Tensor | None = None, out=None, stream=None):
    """Stream form (one word per workgroup, state in LDS); same outputs as decode()."""
    if not llr.is_cuda or llr.dim() != 2 or llr.shape[1] != graph.n:
        raise ValueError("llr must be a cuda tensor of shape [B, n]")
    if llr.dtype not in (torch.float32, torch.float64):
        raise ValueError("llr must be float32 or float64")
    llr = llr.contiguous()
    B = llr.shape[0]
    dev = llr.device
    if out is None:
        hard = torch.empty((B, graph.n), dtype=torch.uint8, device=dev)
        post = torch.empty((B, graph.n), dtype=torch.float32, device=dev)
        iters = torch.empty((B,), dtype=torch.int32, device=dev)
    else:
        hard, post, iters = out
    if workspace is None:
        workspace = torch.empty((256,), dtype=torch.uint8, device=dev)
    flags = LLR_F64 if llr.dtype == torch.float64 else 0
    check("ldpc_decode_stream",
          lib().ldpc_decode_stream(graph.handle, _ptr(llr), B, int(max_iters), int(bool(early_stop)), flags,
                                   _ptr(hard), _ptr(post), _ptr(iters), _ptr(workspace), workspace.numel(),
                                   int(threads), ctypes.c_void_p(stream_handle(stream))))
    return hard, post, iters


def split_workspace_size(graph: Graph, batch: int) -> int:
    out = ctypes.c_size_t()
    check("ldpc_split_workspace_size", lib().ldpc_split_workspace_size(graph.handle, int(batch), ctypes.byref(out)))
    return out.value


def decode_split(graph: Graph, llr: torch.Tensor, max_iters: int, early_stop: bool = True, slices: int = 0,
                 workspace: torch.Tensor | None = None, out=None, stream=None):
    """Split form (each half-iteration one launch over many workgroups per tile); same outputs as decode()."""
    if not llr.is_cuda or llr.dim() != 2 or llr.shape[1] != graph.n:
        raise ValueError("llr must be a cuda tensor of shape [B, n]")
    if llr.dtype not in (torch.float32, torch.float64):
        raise ValueError("llr must be float32 or float64")
    llr = llr.contiguous()
    B = llr.shape[0]
    dev = llr.device
    if out is None:
        hard = torch.empty((B, graph.n), dtype=torch.uint8, device=dev)
        post = torch.empty((B, graph.n), dtype=torch.float32, device=dev)
        iters = torch.empty((B,), dtype=torch.int32, device=dev)
    else:
        hard, post, iters = out
    need = split_workspace_size(graph, B)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty((max(need, 1),), dtype=torch.uint8, device=dev)
    flags = LLR_F64 if llr.dtype == torch.float64 else 0
    check("ldpc_decode_split",
          lib().ldpc_decode_split(graph.handle, _ptr(llr), B, int(max_iters), int(bool(early_stop)), flags,
                                  _ptr(hard), _ptr(post), _ptr(iters), _ptr(workspace), workspace.numel(),
                                  int(slices), ctypes.c_void_p(stream_handle(stream))))
    return hard, post, iters


def syndrome_ok(graph: Graph, hard: torch.Tensor, stream=None) -> torch.Tensor:
    """ldpc_syndrome: uint8 [B], 1 where H z^T = 0 for the decisions hard [B, n] (uint8, nonzero = 1)."""
    if not hard.is_cuda or hard.dtype != torch.uint8 or hard.dim() != 2 or hard.shape[1] != graph.n:
        raise ValueError("hard must be a cuda uint8 tensor of shape [B, n]")
    hard = hard.contiguous()
    ok = torch.empty((hard.shape[0],), dtype=torch.uint8, device=hard.device)
    check("ldpc_syndrome", lib().ldpc_syndrome(graph.handle, _ptr(hard), hard.shape[0], _ptr(ok),
                                               ctypes.c_void_p(stream_handle(stream))))
    return ok
