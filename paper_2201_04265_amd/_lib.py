"""ctypes loader of libldpc_hip.so and the argument types of every exported entry point."""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  -- loads the HIP runtime the library binds to (same soname)

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libldpc_hip.so")

_i32, _i64, _u32, _p = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p
_pi32, _pi64, _psz = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_size_t)

# name -> (argtypes, restype); mirrors include/ldpc.h
SIGNATURES = {
    "ldpc_graph_create": ([_i32, _i32, ctypes.c_int, _p, _p, _i64, ctypes.POINTER(_p)], ctypes.c_int),
    "ldpc_graph_destroy": ([_p], ctypes.c_int),
    "ldpc_graph_info": ([_p, _pi32, _pi32, _pi64, _pi32, _pi32], ctypes.c_int),
    "ldpc_graph_edges": ([_p, _p, _p], ctypes.c_int),
    "ldpc_decode_workspace_size": ([_p, _i32, _u32, _psz], ctypes.c_int),
    "ldpc_decode": ([_p, _p, _i32, _i32, _i32, _u32, _p, _p, _p, _p, ctypes.c_size_t, _p], ctypes.c_int),
    "ldpc_decode_ex": ([_p, _p, _i32, _i32, _i32, _u32, _p, _p, _p, _p, _p, _p, ctypes.c_size_t, _p], ctypes.c_int),
    "ldpc_decode_noalloc": ([_p, _p, _i32, _i32, _i32, _u32, _p, _p, _p, _p], ctypes.c_int),
    "ldpc_decode_config": ([_p, _p, _i32, _i32, _i32, _u32, _p, _p, _p, _p, ctypes.c_size_t, _i32, _p],
                           ctypes.c_int),
    "ldpc_stream_lds_bytes": ([_p, _psz, _pi32], ctypes.c_int),
    "ldpc_decode_stream": ([_p, _p, _i32, _i32, _i32, _u32, _p, _p, _p, _p, ctypes.c_size_t, _i32, _p], ctypes.c_int),
    "ldpc_split_workspace_size": ([_p, _i32, _psz], ctypes.c_int),
    "ldpc_decode_split": ([_p, _p, _i32, _i32, _i32, _u32, _p, _p, _p, _p, ctypes.c_size_t, _i32, _p], ctypes.c_int),
    "ldpc_multi_resolve": ([_p, _i32, _p, _p, _p, _psz], ctypes.c_int),
    "ldpc_decode_multi": ([_p, _i32, _p, _p, _i32, _p, _p, ctypes.c_size_t, _p], ctypes.c_int),
    "ldpc_plan_create_multi": ([_p, _i32, _p, _p, _i32, _p, _p, ctypes.c_size_t, _p, ctypes.POINTER(_p)],
                               ctypes.c_int),
    "ldpc_plan_launch": ([_p, _p], ctypes.c_int),
    "ldpc_plan_destroy": ([_p], ctypes.c_int),
    "ldpc_autotune_multi": ([_p, _i32, _p, _p, _i32, _u32, _p, _p, ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
    "ldpc_unrolled_sizes": ([_p, _i32, _i32, _psz, _psz, _psz], ctypes.c_int),
    "ldpc_unrolled_forward": ([_p, _p, _p, _i32, _i32, _p, _p, ctypes.c_size_t, _p, ctypes.c_size_t, _p],
                              ctypes.c_int),
    "ldpc_unrolled_backward": ([_p, _p, _p, ctypes.c_size_t, _p, _i32, _i32, _p, _p, _p, ctypes.c_size_t, _p],
                               ctypes.c_int),
    "ldpc_encoder_create": ([_p, ctypes.POINTER(_p)], ctypes.c_int),
    "ldpc_encoder_destroy": ([_p], ctypes.c_int),
    "ldpc_encoder_info": ([_p, _pi32, _pi32, _pi32], ctypes.c_int),
    "ldpc_encoder_positions": ([_p, _p, _p], ctypes.c_int),
    "ldpc_encode": ([_p, _p, _i32, _p, _p], ctypes.c_int),
    "ldpc_channel_awgn": ([_p, _i32, _i32, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64, _i64, _u32, _p, _p],
                          ctypes.c_int),
    "ldpc_generate": ([_p, _i32, ctypes.c_uint64, ctypes.c_uint64, _i64, ctypes.c_double, _u32, _p, _p, _p, _p],
                      ctypes.c_int),
    "ldpc_count_errors": ([_p, _p, _p, _i32, _p, _p], ctypes.c_int),
    "ldpc_syndrome": ([_p, _p, _i32, _p, _p], ctypes.c_int),
    "ldpc_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "ldpc_last_error": ([], ctypes.c_char_p),
}

LLR_F64 = 0x1


class LdpcError(RuntimeError):
    def __init__(self, fn: str, status: int, detail: str):
        super().__init__(f"{fn} failed: status {status} ({detail})")
        self.status = status


_lib = None


def lib():
    """The loaded library; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(library_path):
        raise RuntimeError(f"HIP decoder library missing: {library_path} (build it with __graft_entry__.build())")
    h = ctypes.CDLL(library_path)
    for name, (args, res) in SIGNATURES.items():
        f = getattr(h, name)
        f.argtypes = args
        f.restype = res
    _lib = h
    return h


def check(fn: str, status: int) -> None:
    if status != 0:
        h = lib()
        detail = h.ldpc_last_error().decode(errors="replace")
        raise LdpcError(fn, status, f"{h.ldpc_status_string(status).decode()}: {detail}")


def stream_handle(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream
