"""Stream form (one word per workgroup, state in LDS): bit-identical to the plain decoder,
parity with the FP64 oracle, and the LDS limit reported as unsupported."""
import numpy as np
import pytest
import torch

from oracle.parity import assert_parity, compare
from synth import codes, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2201_04265_amd as P

    assert torch.cuda.is_available()
    return P


def both(P, g, llr, T, es=True, threads=0):
    x = torch.from_numpy(np.ascontiguousarray(llr)).cuda()
    a = P.decode(g, x, T, es)
    b = P.decode_stream(g, x, T, es, threads=threads)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in a], [t.cpu().numpy() for t in b]


def same(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_c1_equals_plain_and_oracle(P, oracle_lib):
    code = W.code("c1")
    g = P.Graph.from_code(code)
    wd = W.words("c1", 1, 0, 2.0, 0, 1000, fp32=False)
    a, b = both(P, g, wd.llr, 20)
    same(a, b)
    oh, op, oi, _ = oracle_lib.decode(code, wd.llr, 20, True)
    assert_parity(compare(oh, op, oi, *b, oracle_lib, code, wd.llr, 20))


@pytest.mark.parametrize("ebn0,key", [(1.0, 0), (2.0, 2)])
def test_c2_equals_plain(P, ebn0, key):
    code = W.code("c2")
    g = P.Graph.from_code(code)
    assert P.stream_supported(g)
    wd = W.words("c2", 2, key, ebn0, 0, 3000, fp32=True)
    a, b = both(P, g, wd.llr, 50)
    same(a, b)


@pytest.mark.parametrize("threads", [64, 192, 256, 1024])
def test_workgroup_sizes_agree(P, threads):
    code = W.code("c5")
    g = P.Graph.from_code(code)
    wd = W.words("c5", 5, 0, 1.5, 0, 777, fp32=True)
    a, b = both(P, g, wd.llr, 30, True, threads)
    same(a, b)


def test_fixed_and_zero_iterations(P):
    code = W.code("c5")
    g = P.Graph.from_code(code)
    wd = W.words("c5", 5, 0, 2.0, 0, 300, fp32=True)
    for T, es in ((9, False), (0, False), (0, True)):
        a, b = both(P, g, wd.llr, T, es)
        same(a, b)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("seed", range(3))
def test_irregular_codes(P, oracle_lib, seed, dtype):
    """Runtime-degree codes (mixed degrees inside the groups of 64 checks and variables, n and m
    not multiples of 64) with FP32 and FP64 channel LLRs: bit-identical to the plain decoder."""
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(60, 400))
    m = int(rng.integers(n // 4, n // 2))
    chk, var = [], []
    for c in range(m):
        d = int(rng.integers(2, 25))
        vs = rng.choice(n, size=min(d, n), replace=False)
        chk += [c] * len(vs)
        var += list(vs)
    code = codes.from_edges(m, n, np.array(chk), np.array(var))
    g = P.Graph.from_code(code)
    llr = rng.normal(2.0, 2.0, size=(int(rng.integers(1, 300)), n)).astype(dtype)
    a, b = both(P, g, llr, 15)
    same(a, b)


def test_check_degree_24_with_variable_degrees_above_12(P, oracle_lib):
    """Check degrees up to 24 take the degree-24 class only while every variable degree is at
    most 12; a code with variables of degree 13 to 16 runs the degree-32 class instead, in
    every form: stream and plain bit-identical, both at parity with the oracle."""
    rng = np.random.default_rng(4242)
    n, m = 220, 100
    chk, var = [], []
    for c in range(m):
        vs = set(rng.choice(np.arange(1, n), size=int(rng.integers(10, 22)), replace=False).tolist())
        if c < 14:
            vs.add(0)  # variable 0 in 14 checks
        chk += [c] * len(vs)
        var += sorted(vs)
    code = codes.from_edges(m, n, np.array(chk), np.array(var))
    assert code.row_degrees().max() <= 24 and 13 <= np.bincount(code.indices, minlength=n).max() <= 16
    g = P.Graph.from_code(code)
    llr = rng.normal(2.5, 2.0, size=(150, n)).astype(np.float32)
    a, b = both(P, g, llr, 20)
    same(a, b)
    oh, op, oi, _ = oracle_lib.decode(code, llr, 20, True)
    st = compare(oh, op, oi, a[0], a[1], a[2], oracle_lib, code, llr, 20)
    print(st)
    assert_parity(st, allow_tie_fraction=0.02)


def test_mixed_batch_codes(P):
    """Every mixed-batch code that fits the LDS of a workgroup decodes identically in both forms."""
    for i, name in enumerate(W.C4_CODES):
        code = W.code(name)
        g = P.Graph.from_code(code)
        if not P.stream_supported(g):
            assert code.n >= 5000  # n=16384 and the Z=128 quasi-cyclic code need more than 160 KB
            continue
        wd = W.words(name, 4, 0, float(W.c4_ebn0()[i]), 0, 200, fp32=True, code_key=i)
        a, b = both(P, g, wd.llr, 50)
        same(a, b)


def test_too_large_is_unsupported(P):
    code = W.code("c3")
    g = P.Graph.from_code(code)
    assert not P.stream_supported(g)
    x = torch.zeros((4, code.n), dtype=torch.float32, device="cuda")
    with pytest.raises(P.LdpcError) as e:
        P.decode_stream(g, x, 10)
    assert e.value.status == -5


def test_generic_high_degree_codes_every_workgroup_size(P):
    """Codes outside the fixed degree pairs with check degree 20 (runtime-degree kernel, prefix
    pairs half in the LDS row): 1024- and 512-thread workgroups, both equal to the plain decoder;
    sizes beyond 1024 are refused."""
    rng = np.random.default_rng(77)
    n, m = 300, 40
    chk, var = [], []
    for c in range(m):
        vs = rng.choice(n, size=20, replace=False)
        chk += [c] * 20
        var += list(vs)
    code = codes.from_edges(m, n, np.array(chk), np.array(var))
    g = P.Graph.from_code(code)
    x = torch.from_numpy(rng.normal(2.0, 2.0, size=(9, n)).astype(np.float32)).cuda()
    with pytest.raises(P.LdpcError) as e:
        P.decode_stream(g, x, 5, threads=1088)
    assert e.value.status == -1
    for nt in (1024, 512):
        a, b = both(P, g, x.cpu().numpy(), 12, True, nt)
        same(a, b)


FIXED_PAIRS = {(6, 3), (4, 3), (12, 3), (15, 3), (12, 6), (12, 9)}


def _expected_lds_bytes(code):
    """The documented size: fixed degree pairs keep one row per check (4 bytes per edge);
    other codes interleave 64 degree-sorted checks per group, a group spanning 64 x its
    largest degree floats (the last one up to its last entry)."""
    rd = code.row_degrees()
    cd = np.bincount(code.indices, minlength=code.n)
    if rd.min() == rd.max() and cd.min() == cd.max() and (int(rd[0]), int(cd[0])) in FIXED_PAIRS:
        floats = code.nnz
    else:
        d = np.sort(rd, kind="stable")
        groups = [d[i:i + 64] for i in range(0, len(d), 64)]
        floats = sum(64 * int(gr.max()) for gr in groups[:-1]) + 64 * (int(groups[-1].max()) - 1) + len(groups[-1])
    return (floats * 4 + 15) // 16 * 16 + 80


def _irregular_code(seed, m, n, dmin, dmax):
    rng = np.random.default_rng(seed)
    chk, var = [], []
    for c in range(m):
        vs = rng.choice(n, size=int(rng.integers(dmin, dmax + 1)), replace=False)
        chk += [c] * len(vs)
        var += list(vs)
    return codes.from_edges(m, n, np.array(chk), np.array(var))


def test_lds_bytes_of_the_interleaved_layout(P):
    qc = W.code("c4_5")  # quasi-cyclic, circulant 128: every group has one degree
    assert P.stream_lds_bytes(P.Graph.from_code(qc)) == (qc.nnz * 4 + 15) // 16 * 16 + 80
    for name in ("c2", "c5", "paper_r12"):  # fixed degree pairs
        c = W.code(name)
        assert P.stream_lds_bytes(P.Graph.from_code(c)) == (c.nnz * 4 + 15) // 16 * 16 + 80
    for seed, m, n in ((1, 50, 200), (2, 300, 700), (3, 1500, 4000)):
        c = _irregular_code(seed, m, n, 2, 24)
        got = P.stream_lds_bytes(P.Graph.from_code(c))
        assert got == _expected_lds_bytes(c)
        print(seed, m, n, "edges", c.nnz, "LDS bytes", got, flush=True)
        assert got >= c.nnz * 4


@pytest.mark.parametrize("threads", [0, 256, 1024])
def test_many_check_groups_equal_plain(P, threads):
    """An irregular code with 24 groups of 64 checks (more than one pass of the check phase
    for every workgroup size), mixed degrees 3..20 inside groups at class boundaries."""
    c = _irregular_code(5, 1500, 3000, 3, 20)
    g = P.Graph.from_code(c)
    assert P.stream_supported(g)
    llr = np.random.default_rng(6).normal(1.8, 2.0, size=(150, c.n)).astype(np.float32)
    a, b = both(P, g, llr, 20, True, threads)
    same(a, b)
