"""The degree limits of the kernels (check degree 32, variable degree 16) in every form: plain
against the FP64 oracle, and the stream, split, batched and unrolled (all-ones weights) forms bit
for bit against plain.  Variable degree 17 is refused."""
import numpy as np
import pytest
import torch

from oracle.parity import assert_parity, compare
from synth import codes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2201_04265_amd as P

    assert torch.cuda.is_available()
    return P


def _limit_code(seed=12):
    """Checks of degree 2..32 with several at exactly 32; variable 0 in 16 checks (the maximum)."""
    rng = np.random.default_rng(seed)
    m, n = 48, 400
    chk, var = [], []
    for c in range(m):
        d = 32 if c % 5 == 0 else int(rng.integers(2, 33))
        vs = set(rng.choice(np.arange(1, n), size=d - (1 if c < 16 else 0), replace=False).tolist())
        if c < 16:
            vs.add(0)  # variable 0 joins the first 16 checks
        chk += [c] * len(vs)
        var += sorted(vs)
    code = codes.from_edges(m, n, np.array(chk), np.array(var), "limits")
    deg_v = np.bincount(code.indices, minlength=n)
    assert code.row_degrees().max() == 32 and deg_v.max() == 16
    return code


@pytest.fixture(scope="module")
def limit(P):
    code = _limit_code()
    g = P.Graph.from_code(code)
    rng = np.random.default_rng(3)
    llr = rng.normal(1.5, 2.0, size=(130, code.n)).astype(np.float32)
    return code, g, llr


def _np(o):
    return tuple(t.cpu().numpy() for t in o)


def _same(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_plain_parity_at_the_limits(P, oracle_lib, limit):
    code, g, llr = limit
    assert g.max_check_deg == 32 and g.max_var_deg == 16
    h, p, i = _np(P.decode(g, torch.from_numpy(llr).cuda(), 25, True))
    oh, op, oi, _ = oracle_lib.decode(code, llr, 25, True)
    st = compare(oh, op, oi, h, p, i, oracle_lib, code, llr, 25)
    print(st)
    assert_parity(st, allow_tie_fraction=0.05)


@pytest.mark.parametrize("threads", [0, 512, 1024])
def test_stream_equals_plain_at_the_limits(P, limit, threads):
    code, g, llr = limit
    x = torch.from_numpy(llr).cuda()
    _same(_np(P.decode(g, x, 25, True)), _np(P.decode_stream(g, x, 25, True, threads=threads)))


def test_split_equals_plain_at_the_limits(P, limit):
    code, g, llr = limit
    x = torch.from_numpy(llr).cuda()
    _same(_np(P.decode(g, x, 25, True)), _np(P.decode_split(g, x, 25, True, slices=3)))


def test_batched_equals_plain_at_the_limits(P, limit):
    code, g, llr = limit
    other = codes.from_edges(4, 12, np.repeat(np.arange(4), 3), np.arange(12), "tiny(3 per check)")
    g2 = P.Graph.from_code(other)
    x = torch.from_numpy(llr).cuda()
    y = torch.from_numpy(np.random.default_rng(4).normal(1.0, 2.0, size=(70, 12)).astype(np.float32)).cuda()
    ref = [_np(P.decode(g, x, 25, True)), _np(P.decode(g2, y, 25, True))]
    for shape in (None, P.Shape.make(8, [2, 1], 1)):
        out = P.decode_multi([g, g2], [x, y], 25, True, shape=shape)
        torch.cuda.synchronize()
        for r, o in zip(ref, out):
            _same(r, _np(o))


def test_unrolled_all_ones_equals_plain_at_the_limits(P, limit):
    code, g, llr = limit
    x = torch.from_numpy(llr).cuda()
    T = 6
    w = torch.ones((T, code.nnz), dtype=torch.float32, device="cuda")
    post = P.unrolled_decode(g, x, w)
    _, ref, _ = P.decode(g, x, T, False)
    torch.cuda.synchronize()
    assert torch.equal(post, ref)


def test_variable_degree_17_is_refused(P):
    m, n = 17, 40
    chk = np.repeat(np.arange(m), 2)
    var = np.stack([np.zeros(m, dtype=int), np.arange(1, m + 1)], axis=1).ravel()  # variable 0 in 17 checks
    code = codes.from_edges(m, n, chk, var)
    with pytest.raises(P.LdpcError) as e:
        P.Graph.from_code(code)
    assert e.value.status == -5
