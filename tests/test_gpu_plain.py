"""Parity of the plain HIP decoder (ldpc_decode) against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle.parity import assert_parity, compare
from synth import codes, gf2, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2201_04265_amd as P

    assert torch.cuda.is_available()
    return P


def gpu_decode(P, g, llr, T, es=True, waves=None):
    t = torch.from_numpy(np.ascontiguousarray(llr)).cuda()
    hard, post, iters = P.decode(g, t, T, es, waves=waves)
    torch.cuda.synchronize()
    return hard.cpu().numpy(), post.cpu().numpy(), iters.cpu().numpy()


def test_c1_full_parity(P, oracle_lib):
    """(3,6) n=96 Gallager band, 1000 words, 2.0 dB, FP64 LLRs rounded on ingest, 20 iterations."""
    code = workloads.code("c1")
    wd = workloads.words("c1", 1, 0, 2.0, 0, 1000, fp32=False)
    g = P.Graph.from_code(code)
    oh, op, oi, _ = oracle_lib.decode(code, wd.llr, 20, True)
    gh, gp, gi = gpu_decode(P, g, wd.llr, 20)
    st = compare(oh, op, oi, gh, gp, gi, oracle_lib, code, wd.llr, 20)
    print("C1", st)
    assert_parity(st)
    # BER identical
    assert np.mean(gh != wd.cw) == np.mean(oh != wd.cw) or st["tie_exceptions"] > 0


@pytest.mark.parametrize("waves", [1, 3, 8, 16])
def test_launch_shapes_agree_bitwise(P, waves):
    code = workloads.code("c1")
    wd = workloads.words("c1", 1, 0, 1.5, 0, 300, fp32=True)
    g = P.Graph.from_code(code)
    ref = gpu_decode(P, g, wd.llr, 20, True, waves=8)
    out = gpu_decode(P, g, wd.llr, 20, True, waves=waves)
    for a, b in zip(ref, out):
        assert np.array_equal(a, b)


def test_repeat_is_deterministic(P):
    code = workloads.code("c1")
    wd = workloads.words("c1", 1, 0, 1.0, 0, 640, fp32=True)
    g = P.Graph.from_code(code)
    a = gpu_decode(P, g, wd.llr, 20)
    b = gpu_decode(P, g, wd.llr, 20)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("seed", range(6))
def test_random_irregular_codes_ragged_batches(P, oracle_lib, seed):
    """Irregular codes with odd and even check degrees in [2, 20]; batch not a multiple of 64."""
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(40, 300))
    m = int(rng.integers(n // 4, n // 2))
    chk, var = [], []
    for c in range(m):
        d = int(rng.integers(2, 21))
        vs = rng.choice(n, size=min(d, n), replace=False)
        chk += [c] * len(vs)
        var += list(vs)
    code = codes.from_edges(m, n, np.array(chk), np.array(var))
    B = int(rng.integers(1, 200))
    llr = rng.normal(2.0, 2.0, size=(B, n)).astype(np.float32)  # all-zero word through a noisy channel
    g = P.Graph.from_code(code)
    oh, op, oi, _ = oracle_lib.decode(code, llr, 15, True)
    gh, gp, gi = gpu_decode(P, g, llr, 15)
    st = compare(oh, op, oi, gh, gp, gi, oracle_lib, code, llr, 15)
    print(seed, n, m, B, st)
    assert_parity(st, allow_tie_fraction=0.02)


def _tile_bytes(code):
    """One 64-word tile state: M, E0, E1 [edges][64] and R [n][64] FP32, each 256-byte aligned."""
    al = lambda b: (b + 255) // 256 * 256  # noqa: E731
    return 3 * al(code.nnz * 64 * 4) + al(code.n * 64 * 4)


@pytest.mark.parametrize("states", [1, 2, 3])
def test_small_workspace_reuses_tile_states(P, states):
    """Workgroups take tiles from a counter and reuse their own tile state: a workspace of 256
    bytes plus 1-3 tile states decodes a ragged 10-tile batch (with early stop, so tiles take
    different times) to the same bits as the full-speed workspace, through the C ABI; one byte
    less than a tile state is refused."""
    import ctypes

    code = workloads.code("c1")
    g = P.Graph.from_code(code)
    B = 9 * 64 + 17
    wd = workloads.words("c1", 1, 0, 1.5, 0, B, fp32=True)
    x = torch.from_numpy(wd.llr).cuda()
    ref = P.decode(g, x, 20, True)
    L = P.lib()
    need = ctypes.c_size_t()
    assert L.ldpc_decode_workspace_size(g.handle, B, 0, ctypes.byref(need)) == 0
    assert need.value <= 256 + 10 * _tile_bytes(code)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    for nbytes, ok in ((256 + states * _tile_bytes(code), True), (255 + _tile_bytes(code), False)):
        ws = torch.empty((nbytes,), dtype=torch.uint8, device="cuda")
        h = torch.empty((B, code.n), dtype=torch.uint8, device="cuda")
        po = torch.empty((B, code.n), dtype=torch.float32, device="cuda")
        it = torch.empty((B,), dtype=torch.int32, device="cuda")
        st = L.ldpc_decode(g.handle, p(x), B, 20, 1, 0, p(h), p(po), p(it), p(ws), nbytes, s)
        if not ok:
            assert st == -1
            continue
        assert st == 0, L.ldpc_last_error()
        torch.cuda.synchronize()
        for a, b in zip(ref, (h, po, it)):
            assert torch.equal(a, b)


def test_full_speed_workspace_is_bounded_by_resident_workgroups(P):
    """ldpc_decode_workspace_size: 256 bytes plus one tile state per workgroup the device keeps
    resident (at most one per tile), so the 327 680-word C2 batch asks for its 512 resident
    workgroups' states (5.4 GB), not for its 5120 tiles' (54 GB); a batch of fewer tiles asks
    for exactly its tiles."""
    import ctypes

    code = workloads.code("c2")
    g = P.Graph.from_code(code)
    L = P.lib()
    tb = _tile_bytes(code)
    props = torch.cuda.get_device_properties(0)
    for B, states in ((5 * 65536, None), (3 * 64 + 1, 4)):
        need = ctypes.c_size_t()
        assert L.ldpc_decode_workspace_size(g.handle, B, 0, ctypes.byref(need)) == 0
        assert (need.value - 256) % tb == 0
        got = (need.value - 256) // tb
        if states is None:
            assert 1 <= got <= 4 * props.multi_processor_count < (B + 63) // 64
            print("C2 batch", B, "tile states", got, "bytes", need.value, flush=True)
        else:
            assert got == states


def test_noiseless_and_zero_iterations(P):
    code = workloads.code("c2")
    wd = workloads.words("c2", 2, 0, 2.0, 0, 130, fp32=True)
    g = P.Graph.from_code(code)
    clean = (2.0 * (1.0 - 2.0 * wd.cw.astype(np.float32)) / wd.sigma2).astype(np.float32)
    h, p, i = gpu_decode(P, g, clean, 50)
    assert np.all(i == 0) and np.array_equal(h, wd.cw) and np.array_equal(p, clean)
    h, p, i = gpu_decode(P, g, wd.llr, 0, es=False)
    assert np.all(i == 0) and np.array_equal(p, wd.llr) and np.array_equal(h, (wd.llr <= 0).astype(np.uint8))


def test_empty_batch_is_noop(P):
    code = workloads.code("c1")
    g = P.Graph.from_code(code)
    t = torch.zeros((0, code.n), dtype=torch.float32, device="cuda")
    hard, post, iters = P.decode(g, t, 20)
    assert hard.shape == (0, code.n) and iters.shape == (0,)


def test_empty_batch_every_form(P):
    """An empty batch returns at once in every single-code entry point (no buffer is touched, so
    the binding's zero-size tensors with NULL data may be passed); the adjoint of the unrolled
    decoder still writes its weight gradient, which is zero."""
    import ctypes

    code = workloads.code("c1")
    g = P.Graph.from_code(code)
    for dtype in (torch.float32, torch.float64):
        t = torch.zeros((0, code.n), dtype=dtype, device="cuda")
        for fn in (P.decode_ex, P.decode_stream, P.decode_split):
            hard, post, iters = fn(g, t, 20)[:3]
            assert hard.shape == (0, code.n) and post.shape == (0, code.n) and iters.shape == (0,)
        s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        flags = 1 if dtype == torch.float64 else 0
        assert P.lib().ldpc_decode_noalloc(g.handle, None, 0, 20, 1, flags, None, None, None, s) == 0
    t = torch.zeros((0, code.n), dtype=torch.float32, device="cuda", requires_grad=True)
    w = torch.full((4, g.edges), 0.5, dtype=torch.float32, device="cuda", requires_grad=True)
    post = P.unrolled_decode(g, t, w)
    assert post.shape == (0, code.n)
    post.sum().backward()
    torch.cuda.synchronize()
    assert t.grad.shape == (0, code.n)
    assert torch.count_nonzero(w.grad).item() == 0


def test_fixed_iterations_without_early_stop(P, oracle_lib):
    code = workloads.code("c1")
    wd = workloads.words("c1", 1, 0, 2.0, 0, 200, fp32=True)
    g = P.Graph.from_code(code)
    oh, op, oi, _ = oracle_lib.decode(code, wd.llr, 12, False)
    gh, gp, gi = gpu_decode(P, g, wd.llr, 12, es=False)
    assert np.all(gi == 12)
    assert_parity(compare(oh, op, oi, gh, gp, gi, oracle_lib, code, wd.llr, 12, False))


def test_codeword_sign_flip_symmetry_bitexact(P):
    """Negating the LLRs on a codeword's support negates the posteriors exactly (IEEE negation is exact)."""
    code = workloads.code("c2")
    s = workloads.systematic("c2")
    wd = workloads.words("c2", 2, 1, 1.5, 0, 192, fp32=True)
    c2 = s.encode(np.random.default_rng(1).integers(0, 2, size=(192, s.k), dtype=np.uint8))
    flip = (1.0 - 2.0 * c2).astype(np.float32)
    g = P.Graph.from_code(code)
    h1, p1, i1 = gpu_decode(P, g, wd.llr, 50)
    h2, p2, i2 = gpu_decode(P, g, wd.llr * flip, 50)
    assert np.array_equal(i1, i2)
    assert np.array_equal(p2, p1 * flip)
    nz = p1 != 0
    assert np.array_equal((h2 ^ c2)[nz], h1[nz])


def test_early_stop_matches_first_zero_syndrome(P, oracle_lib):
    code = workloads.code("c1")
    wd = workloads.words("c1", 1, 0, 1.5, 0, 128, fp32=True)
    g = P.Graph.from_code(code)
    _, p_es, i_es = gpu_decode(P, g, wd.llr, 20, True)
    for t in range(0, 21):
        h_t, p_t, _ = gpu_decode(P, g, wd.llr, t, es=False)
        ok = oracle_lib.syndrome_ok(code, h_t) == 1
        first = (i_es == t)
        if t < 20:
            assert np.all(ok[first])  # words stopped before the limit satisfy H z^T = 0 at their t
        assert np.array_equal(p_t[first], p_es[first])  # and report that iteration's posterior
        assert not np.any(ok & (i_es > t))  # no earlier zero syndrome was skipped


@pytest.mark.parametrize("ebn0", workloads.C2["ebn0s"])
def test_c2_full_size_sampled_parity(P, oracle_lib, ebn0):
    """(3,6) n=4096, the full 65536-word batch at 50 iterations, every Eb/N0 point of the sweep;
    512 words checked against the oracle (480 drawn uniformly and the last 32 of the batch),
    whatever their iteration count -- at 1.0 dB most of them run all 50 iterations."""
    code = workloads.code("c2")
    B = workloads.C2["batch"]
    snr_key = workloads.C2["ebn0s"].index(ebn0)
    g = P.Graph.from_code(code)
    wd = workloads.words("c2", 2, snr_key, ebn0, 0, B, fp32=True)
    gh, gp, gi = gpu_decode(P, g, wd.llr, 50)
    rng = np.random.default_rng(int(ebn0 * 10))
    idx = np.unique(np.concatenate([rng.choice(B - 32, 480, replace=False), np.arange(B - 32, B)]))
    oh, op, oi, _ = oracle_lib.decode(code, wd.llr[idx], 50, True)
    st = compare(oh, op, oi, gh[idx], gp[idx], gi[idx], oracle_lib, code, wd.llr[idx], 50)
    print("C2", ebn0, "dB: words", len(idx), "at 50 iterations", int(np.sum(oi == 50)), st,
          "mean iters (whole batch)", gi.mean(), "BER", np.mean(gh != wd.cw), flush=True)
    assert len(idx) >= 512
    assert_parity(st, allow_tie_fraction=0.02)


def test_c3_qc_sampled_parity(P, oracle_lib):
    """QC 22x44 protograph lifted by Z=256 (n=11264), 16384 words at 1.5 dB, 30 iterations; 48 words checked."""
    code = workloads.code("c3")
    B = workloads.C3["batch"]
    g = P.Graph.from_code(code)
    wd = workloads.words("c3", 3, 0, 1.5, 0, B, fp32=True)
    gh, gp, gi = gpu_decode(P, g, wd.llr, 30)
    idx = np.sort(np.random.default_rng(3).choice(B, 48, replace=False))
    oh, op, oi, _ = oracle_lib.decode(code, wd.llr[idx], 30, True)
    st = compare(oh, op, oi, gh[idx], gp[idx], gi[idx], oracle_lib, code, wd.llr[idx], 30)
    print("C3", st, "mean iters", gi.mean(), "BER", np.mean(gh != wd.cw))
    assert_parity(st, allow_tie_fraction=0.05)
