"""ldpc_syndrome (the syndrome test of Eq. 1 on given decisions) against the oracle's, bit for bit:
decoder outputs with satisfied and unsatisfied words, codewords and single flips, bytes other than
0/1 (nonzero = 1), batches of every size modulo the 32-word groups and beyond one launch's
workgroups, codes too long for the 32-word form, and the decoders' own stopping rule."""
import numpy as np
import pytest
import torch

from synth import codes, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2201_04265_amd as P

    assert torch.cuda.is_available()
    return P


def _gpu_ok(P, g, words):
    ok = P.syndrome_ok(g, torch.from_numpy(np.ascontiguousarray(words, dtype=np.uint8)).cuda())
    torch.cuda.synchronize()
    return ok.cpu().numpy()


def _flips(cw, rng):
    """Codewords, and codewords with one, two or three positions flipped."""
    out = [cw]
    for nflip in (1, 2, 3):
        w = cw.copy()
        for b in range(w.shape[0]):
            w[b, rng.choice(w.shape[1], size=nflip, replace=False)] ^= 1
        out.append(w)
    return np.concatenate(out)


@pytest.mark.parametrize("name,cfg,ebn0,B,T", [("c1", 1, 1.0, 1000, 3), ("c2", 2, 2.0, 300, 10),
                                               ("c3", 3, 3.0, 70, 8), ("c4_1", 4, 2.25, 130, 8),
                                               ("c4_5", 4, 3.0, 200, 10)])
def test_equals_oracle_on_decoder_outputs(P, oracle_lib, name, cfg, ebn0, B, T):
    """Hard decisions after a few iterations without early stop (some words satisfy every check,
    some do not), the transmitted codewords, and codewords with 1-3 flips."""
    code = workloads.code(name)
    g = P.Graph.from_code(code)
    key = int(name[3:]) if name.startswith("c4_") else None
    wd = workloads.words(name, cfg, 0, ebn0, 0, B, fp32=True, **({"code_key": key} if key is not None else {}))
    hard, _, _ = P.decode(g, torch.from_numpy(wd.llr).cuda(), T, False)
    words = np.concatenate([hard.cpu().numpy(), _flips(wd.cw, np.random.default_rng(B))])
    ref = oracle_lib.syndrome_ok(code, words)
    got = _gpu_ok(P, g, words)
    n_ok = int(ref[:B].sum())
    print(name, "decoded words passing", n_ok, "of", B)
    assert 0 < n_ok < B  # both outcomes occur among the decoder outputs
    assert np.array_equal(got, ref)
    assert np.all(got[B:2 * B] == 1) and not np.any(got[2 * B:3 * B])


def test_nonzero_bytes_are_ones(P, oracle_lib):
    code = workloads.code("c1")
    g = P.Graph.from_code(code)
    wd = workloads.words("c1", 1, 0, 2.0, 0, 400, fp32=True)
    rng = np.random.default_rng(11)
    words = _flips(wd.cw, rng)
    scaled = words * rng.integers(1, 256, size=words.shape).astype(np.uint8)  # 1 -> any nonzero byte
    got = _gpu_ok(P, g, scaled)
    assert np.array_equal(got, oracle_lib.syndrome_ok(code, (scaled != 0).astype(np.uint8)))
    assert np.array_equal(got, _gpu_ok(P, g, words))


@pytest.mark.parametrize("case", ["n102", "odd_address"])
def test_rows_without_four_byte_alignment(P, oracle_lib, case):
    """Rows read byte by byte: a code with n % 4 != 0, and a batch starting at an odd address."""
    rng = np.random.default_rng(12)
    n = 102 if case == "n102" else 96
    code = codes.gallager_band(n, 3, 6, np.random.default_rng(13), f"band(3,6)n{n}")
    g = P.Graph.from_code(code)
    words = _flips(np.zeros((50, n), dtype=np.uint8), rng)
    words[:50] = rng.integers(0, 2, size=(50, n)).astype(np.uint8)  # random words: almost all fail
    words[0] = 0
    ref = oracle_lib.syndrome_ok(code, words)
    t = torch.from_numpy(words).cuda()
    if case == "odd_address":
        buf = torch.zeros(words.size + 1, dtype=torch.uint8, device="cuda")
        t = buf[1:].view(words.shape)
        t.copy_(torch.from_numpy(words).cuda())
        assert t.data_ptr() % 4 == 1 and t.is_contiguous()
    ok = P.syndrome_ok(g, t).cpu().numpy()
    assert ref[0] == 1 and not np.any(ref[50:100])
    assert np.array_equal(ok, ref)


def test_batch_beyond_one_launch_ragged(P, oracle_lib):
    """More 32-word groups than one launch has workgroups (8192), in a ragged count; short
    batches with ragged last groups; one unsatisfied word among codewords."""
    code = workloads.code("c1")
    g = P.Graph.from_code(code)
    B = 8192 * 32 + 1001
    wd = workloads.words("c1", 1, 0, 1.5, 0, B, fp32=True)
    hard, _, _ = P.decode(g, torch.from_numpy(wd.llr).cuda(), 2, False)
    words = hard.cpu().numpy()
    ref = oracle_lib.syndrome_ok(code, words)
    assert 0 < int(ref.sum()) < B
    assert np.array_equal(_gpu_ok(P, g, words), ref)
    for b in (1, 31, 32, 33, 95):  # ragged last groups of 32 words, offset starts
        assert np.array_equal(_gpu_ok(P, g, words[7:7 + b]), ref[7:7 + b])
    # group boundaries: word 40 alone unsatisfied among codewords, in a batch of 64
    cw = wd.cw[:64].copy()
    cw[40, 3] ^= 1
    want = np.ones(64, dtype=np.uint8)
    want[40] = 0
    assert np.array_equal(_gpu_ok(P, g, cw), want)


@pytest.mark.parametrize("n", [40002, 70002])
def test_long_words(P, oracle_lib, n):
    """Codes too long for 32 words' decision masks in LDS (n > 32768) go one word per workgroup:
    n = 40002 with the word's decisions in LDS, n = 70002 > 65536 gathered from global memory."""
    code = codes.gallager_band(n, 3, 6, np.random.default_rng(5), f"band(3,6)n{n}")
    g = P.Graph.from_code(code)
    rng = np.random.default_rng(6)
    words = _flips(np.zeros((6, code.n), dtype=np.uint8), rng)
    words[0, :] = 1  # all ones: every check of even degree is satisfied
    ref = oracle_lib.syndrome_ok(code, words)
    assert ref[0] == 1 and np.all(ref[1:6] == 1) and not np.any(ref[6:12])
    assert np.array_equal(_gpu_ok(P, g, words), ref)


def test_agrees_with_the_decoders_stopping_rule(P):
    """With early stop, a word that stopped before the limit satisfies every check, and among the
    words at the limit the test finds those that do not; the stream form's decisions (bitwise equal
    to the plain decoder's) give the same results."""
    code = workloads.code("c2")
    g = P.Graph.from_code(code)
    wd = workloads.words("c2", 2, 0, 1.5, 0, 2000, fp32=True)
    x = torch.from_numpy(wd.llr).cuda()
    T = 12
    hard, _, iters = P.decode(g, x, T, True)
    ok = P.syndrome_ok(g, hard).cpu().numpy()
    it = iters.cpu().numpy()
    assert np.all(ok[it < T] == 1)
    assert np.any(it == T) and np.any(ok[it == T] == 0)
    hs, _, _ = P.decode_stream(g, x, T, True)
    assert np.array_equal(P.syndrome_ok(g, hs).cpu().numpy(), ok)


def test_full_sweep_batch_sampled(P, oracle_lib):
    """The (3,6) n=4096 sweep's batch size (327680 words, 1.34 GB of decisions): half codewords
    (zero), half sparse random words; every codeword passes and 512 sampled words equal the oracle.
    Prints the launch time (HIP events, median of 7)."""
    code = workloads.code("c2")
    g = P.Graph.from_code(code)
    B = 327680
    gen = torch.Generator(device="cuda").manual_seed(21)
    hard = (torch.rand((B, code.n), device="cuda", generator=gen) < 0.0005).to(torch.uint8)
    hard[: B // 2].zero_()
    ok = P.syndrome_ok(g, hard)
    ts = []
    for _ in range(7):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        P.syndrome_ok(g, hard)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ms = sorted(ts)[3]
    print(f"syndrome of {B} words, n={code.n}: {ms:.3f} ms, {B * code.n / ms / 1e6:.0f} GB/s of decisions")
    okc = ok.cpu().numpy()
    assert np.all(okc[: B // 2] == 1)
    idx = np.sort(np.random.default_rng(22).choice(B, size=512, replace=False))
    words = hard[torch.from_numpy(idx).cuda()].cpu().numpy()
    ref = oracle_lib.syndrome_ok(code, words)
    assert 0 < int(ref[idx >= B // 2].sum()) < int((idx >= B // 2).sum())  # both outcomes sampled
    assert np.array_equal(okc[idx], ref)


def test_empty_batch_and_bad_shape(P):
    code = workloads.code("c1")
    g = P.Graph.from_code(code)
    assert P.syndrome_ok(g, torch.zeros((0, code.n), dtype=torch.uint8, device="cuda")).shape == (0,)
    with pytest.raises(ValueError):
        P.syndrome_ok(g, torch.zeros((3, code.n + 1), dtype=torch.uint8, device="cuda"))
