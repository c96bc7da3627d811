"""MI355X flooding sum-product LDPC decoding (binding over the C ABI of include/ldpc.h).

Every decoding step runs in the HIP kernels of libldpc_hip.so; this module only
marshals arguments: it passes torch tensors' device pointers and the current
HIP stream to the C entry points.  There is no CPU fallback: if the library is
missing the calls raise.

    g = Graph.from_csr(m, n, indptr, indices)
    hard, post, iters = decode(g, llr, max_iters=50, early_stop=True)
    enc = Encoder(g); msg, cw, llr = enc.generate(batch, sigma2, seed)   # words made on the device
"""
from __future__ import annotations

from ._lib import LdpcError, lib, library_path  # noqa: F401
from .graph import Graph  # noqa: F401
from .decoder import decode, decode_ex, decode_split, decode_stream, split_workspace_size, stream_lds_bytes, stream_supported, syndrome_ok, workspace_size  # noqa: F401,E501
from .multi import SPLIT_AUTO, STREAM_AUTO, Batch, Plan, Shape, decode_multi, fault, tuned_shape  # noqa: F401
from .unrolled import UnrolledBP, unrolled_decode  # noqa: F401
from .encoder import Encoder, channel_awgn  # noqa: F401
