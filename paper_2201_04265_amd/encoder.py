"""Systematic encoder, BPSK/AWGN channel and error counts (ldpc_encoder_* / ldpc_encode /
ldpc_channel_awgn / ldpc_generate / ldpc_count_errors): argument marshalling only."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import LLR_F64, check, lib, stream_handle
from .graph import Graph


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


def _u64(x: int) -> int:
    return int(x) & (2 ** 64 - 1)


class Encoder:
    """Systematic encoder of a graph's code (host reduction of H at construction)."""

    def __init__(self, graph: Graph):
        h = ctypes.c_void_p()
        check("ldpc_encoder_create", lib().ldpc_encoder_create(graph.handle, ctypes.byref(h)))
        self._h = h
        n, k, r = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check("ldpc_encoder_info", lib().ldpc_encoder_info(h, ctypes.byref(n), ctypes.byref(k), ctypes.byref(r)))
        self.n, self.k, self.rank = n.value, k.value, r.value
        info = np.zeros(max(self.k, 1), dtype=np.int32)
        piv = np.zeros(max(self.rank, 1), dtype=np.int32)
        check("ldpc_encoder_positions",
              lib().ldpc_encoder_positions(h, info.ctypes.data_as(ctypes.c_void_p), piv.ctypes.data_as(ctypes.c_void_p)))
        self.info, self.pivots = info[:self.k], piv[:self.rank]

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ldpc_encoder_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 -- interpreter shutdown
            pass

    def encode(self, msg: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Codewords [B, n] (uint8, 0/1) of messages msg [B, k] (cuda uint8, nonzero = 1)."""
        if not msg.is_cuda or msg.dtype != torch.uint8 or msg.dim() != 2 or msg.shape[1] != self.k:
            raise ValueError("msg must be a cuda uint8 tensor of shape [B, k]")
        msg = msg.contiguous()
        B = msg.shape[0]
        cw = out if out is not None else torch.empty((B, self.n), dtype=torch.uint8, device=msg.device)
        check("ldpc_encode", lib().ldpc_encode(self._h, _ptr(msg), B, _ptr(cw), ctypes.c_void_p(stream_handle(stream))))
        return cw

    def generate(self, batch: int, sigma2: float, seed: int, noise_stream: int = 0, first_word: int = 0,
                 f64: bool = False, with_msg: bool = False, device="cuda", out=None, stream=None):
        """Random messages, codewords and LLRs of words first_word .. first_word + batch - 1.

        Returns (msg [B, k] uint8 or None, cw [B, n] uint8, llr [B, n] float32/float64)."""
        if out is None:
            msg = torch.empty((batch, self.k), dtype=torch.uint8, device=device) if with_msg else None
            cw = torch.empty((batch, self.n), dtype=torch.uint8, device=device)
            llr = torch.empty((batch, self.n), dtype=torch.float64 if f64 else torch.float32, device=device)
        else:
            msg, cw, llr = out
        check("ldpc_generate",
              lib().ldpc_generate(self._h, int(batch), _u64(seed), _u64(noise_stream), int(first_word), float(sigma2),
                                  LLR_F64 if f64 else 0, _ptr(msg), _ptr(cw), _ptr(llr),
                                  ctypes.c_void_p(stream_handle(stream))))
        return msg, cw, llr

    def count_errors(self, hard: torch.Tensor, cw: torch.Tensor, counts: torch.Tensor | None = None,
                     stream=None) -> torch.Tensor:
        """Adds [coded bit errors, message bit errors, word errors] to counts (cuda int64 [3])."""
        if hard.shape != cw.shape or hard.dtype != torch.uint8 or cw.dtype != torch.uint8 or hard.shape[1] != self.n:
            raise ValueError("hard and cw must be uint8 [B, n]")
        hard, cw = hard.contiguous(), cw.contiguous()
        if counts is None:
            counts = torch.zeros(3, dtype=torch.int64, device=hard.device)
        check("ldpc_count_errors", lib().ldpc_count_errors(self._h, _ptr(hard), _ptr(cw), hard.shape[0], _ptr(counts),
                                                           ctypes.c_void_p(stream_handle(stream))))
        return counts


def channel_awgn(cw: torch.Tensor, sigma2: float, seed: int, noise_stream: int = 0, first_word: int = 0,
                 f64: bool = False, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """LLRs [B, n] of codewords cw [B, n] (cuda uint8) over BPSK/AWGN with noise variance sigma2."""
    if not cw.is_cuda or cw.dtype != torch.uint8 or cw.dim() != 2:
        raise ValueError("cw must be a cuda uint8 tensor of shape [B, n]")
    cw = cw.contiguous()
    B, n = cw.shape
    llr = out if out is not None else torch.empty((B, n), dtype=torch.float64 if f64 else torch.float32,
                                                  device=cw.device)
    check("ldpc_channel_awgn",
          lib().ldpc_channel_awgn(_ptr(cw), B, n, float(sigma2), _u64(seed), _u64(noise_stream), int(first_word),
                                  LLR_F64 if f64 else 0, _ptr(llr), ctypes.c_void_p(stream_handle(stream))))
    return llr
