"""The Table I workload: Gallager bands n = 1032 with 12 ones per row and 9 / 6 / 3 per column,
1000 vectors each, a preset 10 iterations.  Plain, stream and batched forms against the FP64
oracle and against each other."""
import numpy as np
import pytest
import torch

from oracle.parity import assert_parity, compare
from synth import workloads as W

pytestmark = pytest.mark.gpu
T = W.PAPER["iters"]


@pytest.fixture(scope="module")
def P():
    import paper_2201_04265_amd as P

    assert torch.cuda.is_available()
    return P


@pytest.fixture(scope="module")
def table1(P):
    codes = [W.code(nm) for nm in W.PAPER["codes"]]
    words = [W.paper_words(i) for i in range(len(codes))]
    graphs = [P.Graph.from_code(c) for c in codes]
    llrs = [torch.from_numpy(w.llr).cuda() for w in words]
    return codes, graphs, words, llrs


def _np(o):
    return tuple(t.cpu().numpy() for t in o)


@pytest.mark.parametrize("i", range(3))
def test_fixed_iterations_parity(P, oracle_lib, table1, i):
    codes, graphs, words, llrs = table1
    code, wd = codes[i], words[i]
    plain = P.decode(graphs[i], llrs[i], T, False)
    stream = P.decode_stream(graphs[i], llrs[i], T, False)
    torch.cuda.synchronize()
    a, b = _np(plain), _np(stream)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert np.all(a[2] == T)
    oh, op, oi, _ = oracle_lib.decode(code, wd.llr, T, False)
    st = compare(oh, op, oi, *a, oracle_lib, code, wd.llr, T, False)
    print(code.name, st)
    assert_parity(st)


@pytest.mark.parametrize("i", [1, 2])
def test_early_stop_parity(P, oracle_lib, table1, i):
    """With the syndrome test the rate-1/2 and 3/4 codes stop early on most words at 3 dB."""
    codes, graphs, words, llrs = table1
    code, wd = codes[i], words[i]
    out = _np(P.decode_stream(graphs[i], llrs[i], T, True))
    torch.cuda.synchronize()
    assert out[2].min() < T
    oh, op, oi, _ = oracle_lib.decode(code, wd.llr, T, True)
    st = compare(oh, op, oi, *out, oracle_lib, code, wd.llr, T)
    assert_parity(st)


@pytest.mark.parametrize("es", [False, True])
def test_three_rates_in_one_batched_launch(P, table1, es):
    codes, graphs, words, llrs = table1
    ref = [_np(P.decode(g, x, T, es)) for g, x in zip(graphs, llrs)]
    out = [_np(o) for o in P.decode_multi(graphs, llrs, T, es)]
    torch.cuda.synchronize()
    for r, o in zip(ref, out):
        for x, y in zip(r, o):
            assert np.array_equal(x, y)


def test_single_vector(P, table1):
    """Stream processing in the paper's sense: one vector spread over a whole workgroup."""
    codes, graphs, words, llrs = table1
    for g, x in zip(graphs, llrs):
        a = _np(P.decode(g, x[:1], T, False))
        b = _np(P.decode_stream(g, x[:1], T, False))
        for u, v in zip(a, b):
            assert np.array_equal(u, v)
