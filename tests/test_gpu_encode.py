"""On-device word generation against the oracle: systematic positions and codewords
(bit-exact), Philox message bits (bit-exact), AWGN LLRs (FP64: 1e-13 relative; FP32:
within one unit in the last place, the FP64 values differing only by the last bits of
log / cos / sin), error counts (exact), and the fused generator against the two-step path
(bit-exact)."""
import numpy as np
import pytest
import torch

from oracle import channel as OC
from oracle import encode as OE
from synth import codes, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2201_04265_amd as P

    assert torch.cuda.is_available()
    return P


def _irregular(seed=3, m=60, n=150):
    rng = np.random.default_rng(seed)
    rows = []
    for c in range(m):
        d = int(rng.integers(2, 9))
        rows.append(np.sort(rng.choice(n, size=d, replace=False)))
    H = np.zeros((m, n), dtype=np.uint8)
    for c, r in enumerate(rows):
        H[c, r] = 1
    return codes.from_dense(H, "irregular")


def _code(name):
    if name == "irregular":
        return _irregular()
    if name == "full_rank":  # k = 0: only the zero word
        return codes.from_dense(np.array([[1, 1, 0], [0, 1, 1], [1, 1, 1]], dtype=np.uint8), "full_rank")
    return W.code(name)


CODES = ["c1", "c2", "paper_r14", "c4_2", "c4_5", "irregular", "full_rank"]


@pytest.fixture(scope="module")
def forms():
    return {}


def _form(forms, name):
    if name not in forms:
        code = _code(name)
        forms[name] = (code, OE.systematic(code))
    return forms[name]


def _f32_close(a, b):
    a = np.asarray(a, dtype=np.float32)
    b = np.asarray(b, dtype=np.float32)
    return np.all(np.abs(a.astype(np.float64) - b.astype(np.float64)) <= np.spacing(np.abs(b)).astype(np.float64))


@pytest.mark.parametrize("name", CODES)
def test_positions_and_encoding(P, forms, name):
    code, form = _form(forms, name)
    g = P.Graph.from_code(code)
    enc = P.Encoder(g)
    print(name, "n", enc.n, "k", enc.k, "rank", enc.rank, flush=True)
    assert (enc.n, enc.k, enc.rank) == (code.n, form.k, form.rank)
    assert np.array_equal(enc.info, form.info) and np.array_equal(enc.pivots, form.pivots)
    B = 130  # two full 64-word tiles and a ragged one
    msg = OC.messages(17, 0, B, form.k)
    cw = enc.encode(torch.from_numpy(msg).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(cw.cpu().numpy(), OE.encode(form, msg))
    # nonzero bytes count as ones
    cw2 = enc.encode(torch.from_numpy(msg * 7).cuda())
    assert torch.equal(cw, cw2)


@pytest.mark.parametrize("name,f64", [("c1", True), ("c2", False), ("c4_5", False), ("irregular", True),
                                      ("full_rank", False)])
def test_generate_against_oracle(P, forms, name, f64):
    code, form = _form(forms, name)
    enc = P.Encoder(P.Graph.from_code(code))
    B, seed, stream, first = 150, 220104265, 3, 1000
    s2 = 0.7
    msg, cw, llr = enc.generate(B, s2, seed, stream, first, f64=f64, with_msg=True)
    torch.cuda.synchronize()
    msg, cw, llr = msg.cpu().numpy(), cw.cpu().numpy(), llr.cpu().numpy()
    omsg = OC.messages(seed, first, B, form.k)
    assert np.array_equal(msg, omsg)
    assert np.array_equal(cw, OE.encode(form, omsg))
    ollr = OC.awgn_llr(cw, s2, seed, stream, first, f64=f64)
    if f64:
        assert np.max(np.abs(llr - ollr) / np.maximum(1.0, np.abs(ollr))) <= 1e-13
    else:
        assert _f32_close(llr, ollr)
        print(name, "FP32 LLRs differing from the oracle:", int(np.sum(llr != ollr)), "of", llr.size)


@pytest.mark.parametrize("name", ["c2", "paper_r12", "irregular"])
def test_generate_equals_encode_then_channel(P, forms, name):
    code, form = _form(forms, name)
    enc = P.Encoder(P.Graph.from_code(code))
    msg, cw, llr = enc.generate(200, 0.6, 5, 1, 64 * 7 + 3, with_msg=True)
    cw2 = enc.encode(msg)
    llr2 = P.channel_awgn(cw2, 0.6, 5, 1, 64 * 7 + 3)
    torch.cuda.synchronize()
    assert torch.equal(cw, cw2) and torch.equal(llr, llr2)
    # without the message output, and again: the same draws
    _, cw3, llr3 = enc.generate(200, 0.6, 5, 1, 64 * 7 + 3)
    torch.cuda.synchronize()
    assert torch.equal(cw, cw3) and torch.equal(llr, llr3)


@pytest.mark.parametrize("n,f64", [(5, False), (1031, True), (1031, False), (4096, False)])
def test_channel_ragged_lengths(P, n, f64):
    rng = np.random.default_rng(n)
    B = 77
    cw = rng.integers(0, 2, size=(B, n), dtype=np.uint8)
    first = 2 ** 40 + 11  # high counter bits
    llr = P.channel_awgn(torch.from_numpy(cw).cuda(), 0.55, 99, 7, first, f64=f64)
    torch.cuda.synchronize()
    llr = llr.cpu().numpy()
    ollr = OC.awgn_llr(cw, 0.55, 99, 7, first, f64=f64)
    if f64:
        assert np.max(np.abs(llr - ollr) / np.maximum(1.0, np.abs(ollr))) <= 1e-13
    else:
        assert _f32_close(llr, ollr)


def test_count_errors(P, forms):
    code, form = _form(forms, "c1")
    enc = P.Encoder(P.Graph.from_code(code))
    rng = np.random.default_rng(8)
    B = 301
    cw = rng.integers(0, 2, size=(B, code.n), dtype=np.uint8)
    hard = cw.copy()
    flips = rng.random(size=cw.shape) < 0.01
    hard[flips] ^= 1
    hard[5] = cw[5]  # some clean words
    counts = enc.count_errors(torch.from_numpy(hard).cuda(), torch.from_numpy(cw).cuda())
    torch.cuda.synchronize()
    want = OC.error_counts(hard, cw, form.info)
    assert np.array_equal(counts.cpu().numpy(), want)
    # counts accumulate
    enc.count_errors(torch.from_numpy(hard[:10]).cuda(), torch.from_numpy(cw[:10]).cuda(), counts)
    torch.cuda.synchronize()
    assert np.array_equal(counts.cpu().numpy(), want + OC.error_counts(hard[:10], cw[:10], form.info))
    # rows not 4-byte aligned (one byte into a buffer), and a length not a multiple of 4
    def shifted(a):
        buf = torch.zeros(a.size + 1, dtype=torch.uint8, device="cuda")
        buf[1:] = torch.from_numpy(a.ravel()).cuda()
        return buf[1:].view(a.shape)
    c2 = enc.count_errors(shifted(hard), shifted(cw))
    code_i, form_i = _form(forms, "irregular")
    enc_i = P.Encoder(P.Graph.from_code(code_i))
    cw_i = rng.integers(0, 2, size=(77, code_i.n), dtype=np.uint8)
    hard_i = cw_i ^ (rng.random(size=cw_i.shape) < 0.02).astype(np.uint8)
    c3 = enc_i.count_errors(torch.from_numpy(hard_i).cuda(), torch.from_numpy(cw_i).cuda())
    torch.cuda.synchronize()
    assert code_i.n % 4 != 0
    assert np.array_equal(c2.cpu().numpy(), want)
    assert np.array_equal(c3.cpu().numpy(), OC.error_counts(hard_i, cw_i, form_i.info))


def test_sweep_point_on_device_matches_oracle_pipeline(P, oracle_lib, forms):
    """Generate -> stream decode -> error counts on the device against the same chain in the
    oracle (messages, encoding, channel and FP64 decoding of the oracle's own LLRs)."""
    code, form = _form(forms, "c2")
    g = P.Graph.from_code(code)
    enc = P.Encoder(g)
    B, s2, seed = 256, float(np.float64(1.0) / (2 * 0.5 * 10 ** (2.5 / 10))), 4
    msg, cw, llr = enc.generate(B, s2, seed, 0, 0, with_msg=True)
    hard, post, iters = P.decode_stream(g, llr, 50, True)
    counts = enc.count_errors(hard, cw)
    torch.cuda.synchronize()
    ocw = OE.encode(form, OC.messages(seed, 0, B, form.k))
    ollr = OC.awgn_llr(ocw, s2, seed, 0, 0)
    assert np.array_equal(cw.cpu().numpy(), ocw) and _f32_close(llr.cpu().numpy(), ollr)
    oh, op, oi, _ = oracle_lib.decode(code, ollr, 50, True)
    assert np.array_equal(iters.cpu().numpy(), oi)
    assert np.array_equal(hard.cpu().numpy(), oh)
    assert np.array_equal(counts.cpu().numpy(), OC.error_counts(oh, ocw, form.info))


def test_argument_errors(P, forms):
    code, _ = _form(forms, "c1")
    enc = P.Encoder(P.Graph.from_code(code))
    cw = torch.zeros((4, code.n), dtype=torch.uint8, device="cuda")
    with pytest.raises(P.LdpcError) as e:
        P.channel_awgn(cw, 0.0, 1)
    assert e.value.status == -1
    with pytest.raises(P.LdpcError):
        P.channel_awgn(cw, float("nan"), 1)
    with pytest.raises(P.LdpcError):
        P.channel_awgn(cw, 0.5, 1, 0, -1)
    with pytest.raises(P.LdpcError):
        enc.generate(4, -1.0, 1)
    # empty batches are no-ops
    msg, cw0, llr0 = enc.generate(0, 0.5, 1, with_msg=True)
    assert cw0.shape == (0, code.n)
    assert enc.encode(torch.zeros((0, enc.k), dtype=torch.uint8, device="cuda")).shape == (0, code.n)
