"""Batched persistent form (ldpc_decode_multi, plans, autotuner): bit-exact against the plain
decoder per word, and parity with the FP64 oracle on the mixed six-code batch."""
import numpy as np
import pytest
import torch

from oracle.parity import assert_parity, compare
from synth import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2201_04265_amd as P

    assert torch.cuda.is_available()
    return P


@pytest.fixture(scope="module")
def c4(P):
    """Mixed batch: 4096 words round-robin over six codes, each at its own Eb/N0."""
    names = W.C4_CODES
    counts = W.c4_counts(W.C4["batch"])
    ebn0 = W.c4_ebn0()
    codes = [W.code(nm) for nm in names]
    words = [W.words(nm, 4, 0, float(ebn0[i]), 0, counts[i], fp32=True, code_key=i) for i, nm in enumerate(names)]
    graphs = [P.Graph.from_code(c) for c in codes]
    llrs = [torch.from_numpy(w.llr).cuda() for w in words]
    return codes, graphs, words, llrs, ebn0


def _np(outs):
    return [tuple(t.cpu().numpy() for t in o) for o in outs]


def _plain(P, graphs, llrs, T, es=True):
    res = []
    for g, x in zip(graphs, llrs):
        res.append(P.decode(g, x, T, es))
    torch.cuda.synchronize()
    return _np(res)


def _same(a, b):
    for (h1, p1, i1), (h2, p2, i2) in zip(a, b):
        assert np.array_equal(i1, i2)
        assert np.array_equal(h1, h2)
        assert np.array_equal(p1, p2)


def test_c4_batched_equals_per_code_plain(P, c4):
    codes, graphs, words, llrs, _ = c4
    ref = _plain(P, graphs, llrs, 50)
    out = P.decode_multi(graphs, llrs, 50, True)
    torch.cuda.synchronize()
    _same(ref, _np(out))


def test_c4_oracle_parity_sampled(P, c4, oracle_lib):
    codes, graphs, words, llrs, ebn0 = c4
    out = _np(P.decode_multi(graphs, llrs, 50, True))
    for q, (code, wd) in enumerate(zip(codes, words)):
        idx = np.sort(np.random.default_rng(q).choice(wd.llr.shape[0], 128, replace=False))
        oh, op, oi, _ = oracle_lib.decode(code, wd.llr[idx], 50, True)
        gh, gp, gi = (a[idx] for a in out[q])
        st = compare(oh, op, oi, gh, gp, gi, oracle_lib, code, wd.llr[idx], 50)
        print(code.name, ebn0[q], st)
        assert_parity(st, allow_tie_fraction=0.02)
        # BER of the batched form equals the oracle's on these words
        assert np.array_equal((gh != wd.cw[idx]).sum(), (oh != wd.cw[idx]).sum()) or st["tie_exceptions"]


@pytest.mark.parametrize("waves,slots", [(16, 8), (8, 3), (4, 1), (1, 2)])
def test_refill_equals_plain(P, waves, slots):
    """Few slots for many words: every lane decodes a sequence of words."""
    code = W.code("c2")
    g = P.Graph.from_code(code)
    wd = W.words("c2", 2, 1, 1.5, 0, 2000, fp32=True)
    x = torch.from_numpy(wd.llr).cuda()
    ref = _plain(P, [g], [x], 50)
    out = P.decode_multi([g], [x], 50, True, shape=P.Shape.make(waves, [slots]))
    torch.cuda.synchronize()
    _same(ref, _np(out))


def test_word_order_permutation(P):
    code = W.code("c1")
    g = P.Graph.from_code(code)
    wd = W.words("c1", 1, 0, 1.5, 0, 1500, fp32=True)
    x = torch.from_numpy(wd.llr).cuda()
    order = torch.from_numpy(np.random.default_rng(0).permutation(1500).astype(np.int32)).cuda()
    ref = _plain(P, [g], [x], 20)
    out = P.decode_multi([g], [x], 20, True, shape=P.Shape.make(8, [4]), orders=[order])
    torch.cuda.synchronize()
    _same(ref, _np(out))


def test_fixed_iterations_and_zero_iterations(P):
    code_a, code_b = W.code("c1"), W.code("c5")
    ga, gb = P.Graph.from_code(code_a), P.Graph.from_code(code_b)
    xa = torch.from_numpy(W.words("c1", 1, 0, 2.0, 0, 300, fp32=True).llr).cuda()
    xb = torch.from_numpy(W.words("c5", 5, 0, 2.0, 0, 200, fp32=True).llr).cuda()
    ref = [_plain(P, [ga], [xa], 7, False)[0], _plain(P, [gb], [xb], 0, False)[0]]
    out = P.decode_multi([ga, gb], [xa, xb], [7, 0], False, shape=P.Shape.make(4, [2, 1]))
    torch.cuda.synchronize()
    _same(ref, _np(out))


def test_empty_code_in_batch(P):
    ga, gb = P.Graph.from_code(W.code("c1")), P.Graph.from_code(W.code("c5"))
    xa = torch.from_numpy(W.words("c1", 1, 0, 2.0, 0, 100, fp32=True).llr).cuda()
    xb = torch.zeros((0, gb.n), dtype=torch.float32, device="cuda")
    ref = _plain(P, [ga], [xa], 20)
    out = P.decode_multi([ga, gb], [xa, xb], 20, True)
    torch.cuda.synchronize()
    _same(ref, _np(out)[:1])
    assert out[1][2].numel() == 0


def test_plan_replays_match_eager(P, c4):
    """A captured plan replayed several times, with eager decodes in between, equals the eager result."""
    codes, graphs, words, llrs, _ = c4
    eager = _np(P.decode_multi(graphs, llrs, 50, True))
    batch = P.Batch(graphs, llrs, 50)
    plan = P.Plan(batch, True, P.Shape.make(8))
    other = torch.from_numpy(W.words("c1", 1, 0, 1.0, 0, 500, fp32=True).llr).cuda()
    g1 = P.Graph.from_code(W.code("c1"))
    for rep in range(3):
        for o in batch.outs:
            for t in o:
                t.zero_()
        plan.launch()
        torch.cuda.synchronize()
        _same(eager, _np(batch.outs))
        P.decode(g1, other, 20, True)  # unrelated eager work between replays
        torch.cuda.synchronize()
    plan.close()


def test_autotuner_picks_a_valid_shape(P, tmp_path, monkeypatch):
    monkeypatch.setenv("LDPC_AUTOTUNE_CACHE", str(tmp_path))
    code = W.code("c5")
    g = P.Graph.from_code(code)
    x = torch.from_numpy(W.words("c5", 5, 0, 2.0, 0, 4096, fp32=True).llr).cuda()
    batch = P.Batch([g], [x], 50)
    shape = P.tuned_shape(batch, True, persistent_only=True)
    assert 1 <= shape.waves <= 16 and 1 <= shape.slots[0] <= 4096 and 0 <= shape.lanes <= 64
    assert shape.stream_codes == 0 and shape.split_codes == 0
    assert (tmp_path / "autotune.json").exists()
    again = P.tuned_shape(batch, True, persistent_only=True)  # cache hit
    assert again.waves == shape.waves and again.slots[0] == shape.slots[0] and again.lanes == shape.lanes
    ref = _plain(P, [g], [x], 50)
    _same(ref, _np(batch.run(True, shape)))
    # with the forms tuned too (stream / split / persistent per code): same outputs
    fshape = P.tuned_shape(batch, True)
    _same(ref, _np(batch.run(True, fshape)))
    again = P.tuned_shape(batch, True)
    assert again.stream_codes == fshape.stream_codes and again.split_codes == fshape.split_codes


def test_c4_stream_codes_equal_per_code_plain(P, c4):
    """Codes whose word state fits LDS run in the stream form inside the batched decode;
    the outputs stay bit-identical to per-code plain launches."""
    codes, graphs, words, llrs, _ = c4
    ref = _plain(P, graphs, llrs, 50)
    batch = P.Batch(graphs, llrs, 50)
    shape = P.Shape.make(stream_codes=P.STREAM_AUTO)
    resolved, _ = batch.resolve(shape)
    fits = [P.stream_supported(g) for g in graphs]
    assert fits == [(c.nnz * 4 + 15) // 16 * 16 + 80 + 64 <= 160 * 1024 for c in codes]
    for q in range(len(codes)):
        assert bool((resolved.stream_codes >> q) & 1) == fits[q]
        if fits[q]:
            assert resolved.slots[q] == 0
    _same(ref, _np(batch.run(True, shape)))
    # a fixed-iteration run of only some codes in the stream form
    ref7 = _plain(P, graphs, llrs, 7, False)
    batch7 = P.Batch(graphs, llrs, 7)
    _same(ref7, _np(batch7.run(False, P.Shape.make(8, stream_codes=0b000101))))


def test_plan_with_stream_codes_replays_match_eager(P, c4):
    codes, graphs, words, llrs, _ = c4
    eager = _plain(P, graphs, llrs, 50)
    batch = P.Batch(graphs, llrs, 50)
    plan = P.Plan(batch, True, P.Shape.make(stream_codes=P.STREAM_AUTO))
    for rep in range(3):
        for o in batch.outs:
            for t in o:
                t.zero_()
        plan.launch()
        torch.cuda.synchronize()
        _same(eager, _np(batch.outs))
        P.decode(graphs[0], llrs[0], 20, True)  # unrelated eager work between replays
        torch.cuda.synchronize()
    plan.close()


def test_stream_code_that_does_not_fit_is_unsupported(P, c4):
    codes, graphs, words, llrs, _ = c4
    big = [i for i, g in enumerate(graphs) if not P.stream_supported(g)]
    assert big  # the n=16384 code
    batch = P.Batch(graphs, llrs, 50)
    with pytest.raises(P.LdpcError) as e:
        batch.run(True, P.Shape.make(stream_codes=1 << big[0]))
    assert e.value.status == -5


def test_orders_with_stream_codes(P, c4):
    """A word order only changes the schedule: with some codes in the stream form (which takes
    words in its own order) the outputs still equal per-code plain decoding."""
    codes, graphs, words, llrs, _ = c4
    ref = _plain(P, graphs, llrs, 30)
    orders = [torch.randperm(x.shape[0], generator=torch.Generator().manual_seed(q)).to(torch.int32).cuda()
              for q, x in enumerate(llrs)]
    out = P.decode_multi(graphs, llrs, 30, True, shape=P.Shape.make(stream_codes=P.STREAM_AUTO), orders=orders)
    torch.cuda.synchronize()
    _same(ref, _np(out))


@pytest.mark.parametrize("span,slots,lanes,refill", [(4, 4, 64, 1), (3, 5, 32, 4), (8, 2, 16, 1), (2, 11, 64, 64)])
def test_group_slots_equal_plain(P, span, slots, lanes, refill):
    """Slots shared by several workgroups (phases split over them, barriers in global memory)
    give the plain decoder's outputs bit for bit, with refill, narrow slots and batched refills."""
    code = W.code("c2")
    g = P.Graph.from_code(code)
    wd = W.words("c2", 2, 3, 1.5, 0, 700, fp32=True)
    x = torch.from_numpy(wd.llr).cuda()
    ref = _plain(P, [g], [x], 50)
    batch = P.Batch([g], [x], 50)
    sh = P.Shape.make(8, [slots], refill, lanes=lanes, span=[span])
    r, _ = batch.resolve(sh)
    assert r.span[0] == span and r.slots[0] == slots
    ws = batch.workspace(sh)
    batch.run(True, sh, ws)
    torch.cuda.synchronize()
    _same(ref, _np(batch.outs))
    assert P.fault(ws) == 0


def test_group_slots_mixed_codes_fixed_iterations(P):
    """Two codes of different degree profiles (the mixed kernel), group slots, no early stop,
    one code at zero iterations; the same workspace used twice."""
    code_a, code_b = W.code("c1"), W.code("c3")
    ga, gb = P.Graph.from_code(code_a), P.Graph.from_code(code_b)
    xa = torch.from_numpy(W.words("c1", 1, 0, 2.0, 0, 300, fp32=True).llr).cuda()
    xb = torch.from_numpy(W.words("c3", 3, 0, 1.5, 0, 70, fp32=True).llr).cuda()
    for T in ((7, 3), (0, 2)):
        ref = [_plain(P, [ga], [xa], T[0], False)[0], _plain(P, [gb], [xb], T[1], False)[0]]
        batch = P.Batch([ga, gb], [xa, xb], list(T))
        sh = P.Shape.make(16, [2, 2], span=[3, 6])
        ws = batch.workspace(sh)
        batch.run(False, sh, ws)
        torch.cuda.synchronize()
        _same(ref, _np(batch.outs))
        assert P.fault(ws) == 0


def test_group_slots_beyond_capacity_rejected(P):
    """A code's slots are capped at what the GPU holds resident; explicit group slots of several
    codes that the GPU cannot hold resident at once are refused before any launch."""
    g = P.Graph.from_code(W.code("c1"))
    x = torch.from_numpy(W.words("c1", 1, 0, 2.0, 0, 64 * 64, fp32=True).llr).cuda()
    batch = P.Batch([g], [x], 20)
    r, _ = batch.resolve(P.Shape.make(16, [64], span=[64]))
    assert r.span[0] == 64 and 1 <= r.slots[0] < 64  # 16-wave workgroups: at most a few resident per CU
    cap = r.slots[0] * 64
    two = P.Batch([g, g], [x, x], 20)
    with pytest.raises(Exception, match="resident"):
        two.resolve(P.Shape.make(16, [r.slots[0], r.slots[0]], span=[64, 64]))
    assert cap >= 64


def test_automatic_group_slots_for_few_words_of_a_long_code(P):
    """A batch of few words of a long code gets group slots automatically; outputs equal plain."""
    code = W.code("c3")
    g = P.Graph.from_code(code)
    x = torch.from_numpy(W.words("c3", 3, 1, 1.5, 0, 130, fp32=True).llr).cuda()
    batch = P.Batch([g], [x], 30)
    r, _ = batch.resolve(P.Shape.make(16))
    assert r.slots[0] == 3 and r.span[0] > 1
    ref = _plain(P, [g], [x], 30)
    ws = batch.workspace(P.Shape.make(16))
    batch.run(True, P.Shape.make(16), ws)
    torch.cuda.synchronize()
    _same(ref, _np(batch.outs))
    assert P.fault(ws) == 0


def test_group_barrier_failure_is_reported_and_recovered(P, monkeypatch):
    """The group barriers' bounded wait forced to give up at once (a limit of 0 polls, set from
    the host): the launch still ends, the workspace's fault word reports it, and the next launch
    with the default limit is correct again."""
    code = W.code("c2")
    g = P.Graph.from_code(code)
    x = torch.from_numpy(W.words("c2", 2, 4, 2.0, 0, 300, fp32=True).llr).cuda()
    ref = _plain(P, [g], [x], 50)
    batch = P.Batch([g], [x], 50)
    sh = P.Shape.make(8, [3], span=[4])
    ws = batch.workspace(sh)
    monkeypatch.setenv("LDPC_GROUP_SPIN_LIMIT", "0")
    batch.run(True, sh, ws)
    torch.cuda.synchronize()
    assert P.fault(ws) != 0
    monkeypatch.delenv("LDPC_GROUP_SPIN_LIMIT")
    batch.run(True, sh, ws)
    torch.cuda.synchronize()
    assert P.fault(ws) == 0
    _same(ref, _np(batch.outs))
