"""ORACLE -- test infrastructure only.

A plain, slow, FP64 CPU reference for what the GPU decoder computes.  Only the
tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg may
import it; the decoder package never does, and the two share no code.

* ``decode``      -- flooding sum-product (Eqs. 4-8, Algorithm 1's flooding
                     order) with syndrome early stop, C (spa.c), FP64;
* ``decode_ex``   -- the same from a given c->v state, returning the final state
                     (one-step checks); ``store32=True`` selects the build of the same
                     source that rounds every stored value to FP32 (spa.c header);
* ``unrolled``    -- the per-edge-weighted unrolled form (C, FP64);
* ``syndrome_ok`` -- H z^T = 0 test (Eq. 1);
* ``bitwise_map`` -- exact bitwise MAP by enumerating every codeword (map.py);
* ``grad``        -- torch FP64 reference gradient and finite differences (grad.py);
* ``encode``      -- systematic GF(2) encoder from H (Eqs. 1-3), dense and direct (encode.py);
* ``channel``     -- Philox4x64-10 message bits and Box-Muller AWGN LLRs (Eq. 4), numpy (channel.py).

Every function takes a code as any object with ``m, n, indptr, indices`` (CSR
of H, column indices ascending within each row).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_spa.so")
_SO32 = os.path.join(_HERE, "_spa_store32.so")  # same source, stored values rounded to FP32
_lib = None
_lib32 = None


def build() -> str:
    """Compile spa.c with gcc into oracle/_spa.so (plain -O2, no fast-math, no FMA), and the
    FP32-storage build of the same source into oracle/_spa_store32.so."""
    src = os.path.join(_HERE, "spa.c")
    for so, extra in ((_SO, []), (_SO32, ["-DORACLE_STORE32"])):
        tmp = so + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared"] + extra +
                              ["-o", tmp, src, "-lm", "-lpthread"])
        os.replace(tmp, so)
    return _SO


def _open(path):
    lib = ctypes.CDLL(path)
    i32, i64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.oracle_decode.argtypes = [i32, i32, p, p, p, i64, i32, i32, i32, p, p, p, p]
    lib.oracle_decode.restype = ctypes.c_int
    lib.oracle_decode_ex.argtypes = [i32, i32, p, p, p, i64, i32, i32, i32, p, p, p, p, p, p]
    lib.oracle_decode_ex.restype = ctypes.c_int
    lib.oracle_unrolled.argtypes = [i32, i32, p, p, p, i64, i32, p, i32, p]
    lib.oracle_unrolled.restype = ctypes.c_int
    lib.oracle_syndrome_ok.argtypes = [i32, i32, p, p, p, i64, p]
    lib.oracle_syndrome_ok.restype = ctypes.c_int
    return lib


def _load(store32: bool = False):
    global _lib, _lib32
    if store32:
        if _lib32 is None:
            if not os.path.exists(_SO32):
                build()
            _lib32 = _open(_SO32)
        return _lib32
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    _lib = _open(_SO)
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr(code):
    rp = np.ascontiguousarray(code.indptr, dtype=np.int32)
    ci = np.ascontiguousarray(code.indices, dtype=np.int32)
    return rp, ci


def default_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def decode(code, llr, max_iters: int, early_stop: bool = True, nthreads: int | None = None):
    """FP64 flooding sum-product.  Returns (hard u8 [B,n], post f64 [B,n], iters i32 [B], converged u8 [B])."""
    lib = _load()
    llr = np.ascontiguousarray(np.asarray(llr, dtype=np.float64))
    if llr.ndim == 1:
        llr = llr[None, :]
    B, n = llr.shape
    assert n == code.n
    rp, ci = _csr(code)
    hard = np.zeros((B, n), dtype=np.uint8)
    post = np.zeros((B, n), dtype=np.float64)
    iters = np.zeros(B, dtype=np.int32)
    conv = np.zeros(B, dtype=np.uint8)
    rc = lib.oracle_decode(code.m, code.n, _ptr(rp), _ptr(ci), _ptr(llr), B, int(max_iters), int(bool(early_stop)),
                           int(nthreads or default_threads()), _ptr(hard), _ptr(post), _ptr(iters), _ptr(conv))
    if rc:
        raise RuntimeError(f"oracle_decode failed ({rc})")
    return hard, post, iters, conv


def decode_ex(code, llr, max_iters: int, early_stop: bool = True, init_cv=None, store32: bool = False,
              nthreads: int | None = None):
    """Flooding sum-product from the c->v state init_cv [B, nnz] (CSR edge order; None = zeros).

    Returns (hard, post, iters, converged, final_cv [B, nnz] f64): final_cv holds the c->v
    messages of each word's last iteration (init_cv, or zeros, when it stops at 0).
    store32 selects the FP32-storage build of the same source.
    """
    lib = _load(store32)
    llr = np.ascontiguousarray(np.asarray(llr, dtype=np.float64))
    if llr.ndim == 1:
        llr = llr[None, :]
    B, n = llr.shape
    assert n == code.n
    rp, ci = _csr(code)
    nnz = int(rp[-1])
    if init_cv is not None:
        init_cv = np.ascontiguousarray(np.asarray(init_cv, dtype=np.float64))
        assert init_cv.shape == (B, nnz)
    hard = np.zeros((B, n), dtype=np.uint8)
    post = np.zeros((B, n), dtype=np.float64)
    iters = np.zeros(B, dtype=np.int32)
    conv = np.zeros(B, dtype=np.uint8)
    fin = np.zeros((B, nnz), dtype=np.float64)
    rc = lib.oracle_decode_ex(code.m, code.n, _ptr(rp), _ptr(ci), _ptr(llr), B, int(max_iters),
                              int(bool(early_stop)), int(nthreads or default_threads()),
                              _ptr(init_cv) if init_cv is not None else None, _ptr(fin), _ptr(hard), _ptr(post),
                              _ptr(iters), _ptr(conv))
    if rc:
        raise RuntimeError(f"oracle_decode_ex failed ({rc})")
    return hard, post, iters, conv, fin


def unrolled(code, llr, w):
    """Unrolled weighted form, T = w.shape[0] iterations.  Returns the FP64 posterior [B, n]."""
    lib = _load()
    llr = np.ascontiguousarray(np.asarray(llr, dtype=np.float64))
    if llr.ndim == 1:
        llr = llr[None, :]
    w = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
    T = w.shape[0]
    assert w.shape[1:] == (code.nnz,) if hasattr(code, "nnz") else True
    B, n = llr.shape
    rp, ci = _csr(code)
    post = np.zeros((B, n), dtype=np.float64)
    rc = lib.oracle_unrolled(code.m, code.n, _ptr(rp), _ptr(ci), _ptr(llr), B, T, _ptr(w) if T else None,
                             int(default_threads()), _ptr(post))
    if rc:
        raise RuntimeError(f"oracle_unrolled failed ({rc})")
    return post


def syndrome_ok(code, words) -> np.ndarray:
    """ok[b] = 1 iff H z_b^T = 0 over GF(2)."""
    lib = _load()
    words = np.ascontiguousarray(np.asarray(words, dtype=np.uint8))
    if words.ndim == 1:
        words = words[None, :]
    rp, ci = _csr(code)
    ok = np.zeros(words.shape[0], dtype=np.uint8)
    lib.oracle_syndrome_ok(code.m, code.n, _ptr(rp), _ptr(ci), _ptr(words), words.shape[0], _ptr(ok))
    return ok


def bce_loss(post, cw) -> float:
    """Mean over (word, bit) of BCE(sigmoid(-L), c) = c*softplus(L) + (1-c)*softplus(-L), FP64."""
    L = np.asarray(post, dtype=np.float64)
    c = np.asarray(cw, dtype=np.float64)
    sp = lambda x: np.logaddexp(0.0, x)  # noqa: E731
    return float(np.mean(c * sp(L) + (1.0 - c) * sp(-L)))


from .map import bitwise_map  # noqa: E402,F401
