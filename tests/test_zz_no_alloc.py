"""ldpc_decode_noalloc (no device allocation, fixed scratch array) against ldpc_decode, through
the C ABI: bit-identical outputs on two calls in a row, the second with a smaller batch; a
clear error for a batch whose tile state exceeds the fixed array; and any batch of a code
small enough that the resident workgroups' tile states fit the array (tiles taken in turn)."""
import ctypes

import numpy as np
import pytest
import torch

from synth import codes, workloads

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 64 << 20  # LDPC_NOALLOC_SCRATCH_BYTES


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _outs(B, n):
    return (torch.empty((B, n), dtype=torch.uint8, device="cuda"),
            torch.empty((B, n), dtype=torch.float32, device="cuda"),
            torch.empty((B,), dtype=torch.int32, device="cuda"))


def _reference(L, g, x, T, es, f64):
    B = x.shape[0]
    need = ctypes.c_size_t()
    assert L.ldpc_decode_workspace_size(g.handle, B, 1 if f64 else 0, ctypes.byref(need)) == 0
    ws = torch.empty((max(need.value, 1),), dtype=torch.uint8, device="cuda")
    h, p, i = _outs(B, g.n)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = L.ldpc_decode(g.handle, _p(x), B, T, int(es), 1 if f64 else 0, _p(h), _p(p), _p(i), _p(ws), ws.numel(), s)
    assert st == 0, L.ldpc_last_error()
    return h, p, i


def _noalloc(L, g, x, T, es, f64):
    B = x.shape[0]
    h, p, i = _outs(B, g.n)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = L.ldpc_decode_noalloc(g.handle, _p(x), B, T, int(es), 1 if f64 else 0, _p(h), _p(p), _p(i), s)
    assert st == 0, L.ldpc_last_error()
    return h, p, i


@pytest.mark.parametrize("name,cfg,snr,B1,B2,T,f64", [
    ("c2", 2, 1.5, 384, 130, 50, False),   # the (3,6) n=4096 code at the array's limit, then a ragged batch
    ("c1", 1, 2.0, 1000, 77, 20, True),    # n=96 with FP64 LLRs
])
def test_noalloc_equals_decode_twice(name, cfg, snr, B1, B2, T, f64):
    import paper_2201_04265_amd as P

    L = P.lib()
    code = workloads.code(name)
    g = P.Graph.from_code(code)
    wd = workloads.words(name, cfg, 0, snr, 0, B1, fp32=not f64)
    x1 = torch.from_numpy(wd.llr).cuda()
    x2 = x1[:B2].contiguous()
    for x in (x1, x2):  # second call smaller: stale state from the first must not leak
        print(name, "batch", x.shape[0], flush=True)
        ref = _reference(L, g, x, T, True, f64)
        got = _noalloc(L, g, x, T, True, f64)
        torch.cuda.synchronize()
        for a, b in zip(ref, got):
            assert torch.equal(a, b)


def test_noalloc_rejects_batch_above_the_array():
    import paper_2201_04265_amd as P

    L = P.lib()
    code = workloads.code("c2")
    g = P.Graph.from_code(code)
    B = 385  # 7 tiles of the n=4096 code: 7 x 10.5 MB > 64 MiB
    x = torch.zeros((B, code.n), dtype=torch.float32, device="cuda")
    h, p, i = _outs(B, code.n)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = L.ldpc_decode_noalloc(g.handle, _p(x), B, 50, 1, 0, _p(h), _p(p), _p(i), s)
    assert st == -1
    assert b"scratch" in L.ldpc_last_error()


def test_noalloc_small_code_any_batch():
    """A (3,6) n=48 code: 512 resident tile states of 123 kB fit the 64 MiB array, so a batch of
    700 tiles (more than the array or the GPU holds at once) is accepted; workgroups take the
    tiles in turn and the outputs equal ldpc_decode's."""
    import paper_2201_04265_amd as P

    L = P.lib()
    code = codes.gallager_band(48, 3, 6, codes.rng_for(77, 0), "band(3,6)n48")
    g = P.Graph.from_code(code)
    B = 700 * 64 - 5
    rng = np.random.default_rng(78)
    x = torch.from_numpy(rng.normal(1.2, 1.6, size=(B, code.n)).astype(np.float32)).cuda()
    print("n=48 batch", B, flush=True)
    ref = _reference(L, g, x, 30, True, False)
    got = _noalloc(L, g, x, 30, True, False)
    torch.cuda.synchronize()
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
