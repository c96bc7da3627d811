"""Differentiable unrolled decoder: torch.autograd.Function over ldpc_unrolled_forward /
ldpc_unrolled_backward (hand-written HIP forward and adjoint; no torch arithmetic)."""
from __future__ import annotations

import ctypes

import torch

from ._lib import check, lib, stream_handle
from .graph import Graph


def _p(t: torch.Tensor | None) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


def sizes(graph: Graph, batch: int, T: int):
    ck, fw, bw = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    check("ldpc_unrolled_sizes", lib().ldpc_unrolled_sizes(graph.handle, int(batch), int(T), ctypes.byref(ck),
                                                           ctypes.byref(fw), ctypes.byref(bw)))
    return ck.value, fw.value, bw.value


def _buf(nbytes, dev):
    return torch.empty((max(int(nbytes), 256),), dtype=torch.uint8, device=dev)


class UnrolledBP(torch.autograd.Function):
    """posterior = UnrolledBP.apply(llr [B, n] f32, w [T, edges] f32, graph).

    The forward keeps the per-iteration checkpoints of the v->c messages on the
    context; the backward recomputes check messages from them."""

    @staticmethod
    def forward(ctx, llr, w, graph):
        if not (llr.is_cuda and llr.dtype == torch.float32 and llr.dim() == 2 and llr.shape[1] == graph.n):
            raise ValueError("llr must be a cuda float32 tensor [B, n]")
        if not (w.is_cuda and w.dtype == torch.float32 and w.dim() == 2 and w.shape[1] == graph.edges):
            raise ValueError("w must be a cuda float32 tensor [T, edges]")
        llr = llr.contiguous()
        w = w.contiguous()
        B, T = llr.shape[0], w.shape[0]
        ck, fw, _ = sizes(graph, B, T)
        ckpt = _buf(ck, llr.device)
        ws = _buf(fw, llr.device)
        post = torch.empty_like(llr)
        check("ldpc_unrolled_forward",
              lib().ldpc_unrolled_forward(graph.handle, _p(llr), _p(w), B, T, _p(post), _p(ckpt), ckpt.numel(),
                                          _p(ws), ws.numel(), ctypes.c_void_p(stream_handle())))
        ctx.graph = graph
        ctx.ckpt = ckpt
        ctx.shape = (B, T)
        ctx.save_for_backward(w)
        return post

    @staticmethod
    def backward(ctx, grad_post):
        (w,) = ctx.saved_tensors
        graph = ctx.graph
        B, T = ctx.shape
        gp = grad_post.contiguous().to(torch.float32)
        _, _, bw = sizes(graph, B, T)
        ws = _buf(bw, gp.device)
        grad_llr = torch.empty_like(gp)
        grad_w = torch.empty_like(w)
        check("ldpc_unrolled_backward",
              lib().ldpc_unrolled_backward(graph.handle, _p(w), _p(ctx.ckpt), ctx.ckpt.numel(), _p(gp), B, T,
                                           _p(grad_llr), _p(grad_w), _p(ws), ws.numel(),
                                           ctypes.c_void_p(stream_handle())))
        return grad_llr, grad_w, None


def unrolled_decode(graph: Graph, llr: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
    """Posterior LLRs of T = w.shape[0] weighted flooding iterations, differentiable in llr and w."""
    return UnrolledBP.apply(llr, w, graph)
