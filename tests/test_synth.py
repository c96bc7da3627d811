"""Input generator checks: code constructions, the GF(2) systematic encoder, the channel."""
import numpy as np
import pytest

from conftest import read_golden
from synth import channel, codes, gf2, workloads


def _dense_syndrome(H, words):
    return (np.asarray(words, dtype=np.int64) @ np.asarray(H, dtype=np.int64).T) & 1


def test_fig1_matrix_and_edges():
    g = read_golden("fig1_H.txt")
    H = g[None]
    code = codes.fig1_matrix()
    assert np.array_equal(code.dense(), H)
    # the drawn Tanner graph has an edge (v, c) exactly where H[c, v] = 1
    drawn = np.zeros_like(H)
    for v, c in g["edges"]:
        drawn[c - 1, v - 1] = 1
    assert np.array_equal(drawn, H)
    assert np.all(code.col_degrees() == 2) and np.all(code.row_degrees() == 4)


def test_fig1_rank_and_codebook_by_brute_force():
    code = codes.fig1_matrix()
    H = code.dense()
    s = gf2.systematic(code)
    assert s.rank == gf2.gf2_rank(H) == 3 and s.k == 5
    allw = ((np.arange(256)[:, None] >> np.arange(8)[None, :]) & 1).astype(np.uint8)
    cws = allw[np.all(_dense_syndrome(H, allw) == 0, axis=1)]
    assert len(cws) == 32  # 2^k words satisfy H p^T = 0 (Eq. 1)
    G = s.generator()
    enc = s.encode(((np.arange(32)[:, None] >> np.arange(5)[None, :]) & 1).astype(np.uint8))
    assert {tuple(r) for r in enc} == {tuple(r) for r in cws}
    assert np.all((H.astype(int) @ G.T.astype(int)) % 2 == 0)  # Eq. 2


def test_fig2_worked_encoding():
    g = read_golden("fig2_encode.txt")
    m, G, p = g["m"][0], g["G"], g["p"][0]
    assert np.array_equal((m @ G) % 2, p)
    # G is in [I_4 : P] form: the information bits are copied, the parities are m P
    assert np.array_equal(G[:, :4], np.eye(4, dtype=int))
    # the systematic encoder's own [I | P] layout reproduces the printed word
    s = gf2.Systematic(n=8, rank=4, k=4, pivots=np.arange(4, 8), info=np.arange(4), A=G[:, 4:].T.astype(np.uint8))
    assert np.array_equal(s.encode(m[None, :])[0], p)
    assert np.array_equal(s.generator(), G)
    # not a codeword of Fig. 1's H (the caption calls G random)
    assert np.any(_dense_syndrome(codes.fig1_matrix().dense(), p[None, :]))


@pytest.mark.parametrize("n,dv,dc", [(96, 3, 6), (1024, 3, 4), (1032, 9, 12), (1032, 3, 12)])
def test_gallager_band(n, dv, dc):
    code = codes.gallager_band(n, dv, dc, np.random.default_rng(n + dv))
    assert code.m == n * dv // dc
    assert np.all(code.col_degrees() == dv) and np.all(code.row_degrees() == dc)
    H = code.dense()
    rb = n // dc
    for b in range(dv):  # every band partitions the columns
        assert np.all(H[b * rb:(b + 1) * rb].sum(axis=0) == 1)
    assert np.array_equal(H[:rb], np.kron(np.eye(rb, dtype=np.uint8), np.ones((1, dc), dtype=np.uint8)))
    # a band-structured matrix has dependent rows: the bands sum to the all-ones row each
    assert gf2.gf2_rank(H) <= code.m - dv + 1


@pytest.mark.parametrize("n,dv,dc", [(128, 3, 6), (4096, 3, 6), (2048, 3, 12), (4000, 3, 15)])
def test_socket_regular_girth6(n, dv, dc):
    code = codes.socket_regular(n, dv, dc, np.random.default_rng(7 + n), girth6=True)
    assert np.all(code.col_degrees() == dv) and np.all(code.row_degrees() == dc)
    assert codes.girth_at_least_6(code)
    key = np.repeat(np.arange(code.m), code.row_degrees()) * n + code.indices
    assert np.unique(key).size == key.size


def test_qc_lift_structure():
    Z = 16
    base = codes.qc_protograph(22, 44, Z, np.random.default_rng(3))
    w = (base >= 0).sum(axis=0)
    assert np.all((w >= 3) & (w <= 10)) and np.all((base >= 0).sum(axis=1) >= 2)
    code = codes.qc_lift(base, Z)
    H = code.dense()
    for i in range(22):
        for j in range(44):
            blk = H[i * Z:(i + 1) * Z, j * Z:(j + 1) * Z]
            if base[i, j] < 0:
                assert not blk.any()
            else:
                expect = np.roll(np.eye(Z, dtype=np.uint8), int(base[i, j]), axis=1)
                assert np.array_equal(blk, expect)  # row r -> column (r + s) mod Z


def test_encoder_null_space_and_rank():
    for code in [codes.socket_regular(512, 3, 6, np.random.default_rng(1)),
                 codes.gallager_band(96, 3, 6, np.random.default_rng(2)),
                 codes.qc_lift(codes.qc_protograph(22, 44, 8, np.random.default_rng(4)), 8)]:
        s = gf2.systematic(code)
        H = code.dense()
        G = s.generator()
        assert s.rank == gf2.gf2_rank(H)
        assert gf2.gf2_rank(G) == s.k == code.n - s.rank
        assert not np.any((H.astype(np.int64) @ G.T.astype(np.int64)) & 1)  # H G^T = 0 (Eq. 2)
        msg = np.random.default_rng(5).integers(0, 2, size=(64, s.k), dtype=np.uint8)
        cw = s.encode(msg)
        assert not np.any(_dense_syndrome(H, cw))
        assert np.array_equal(cw, (msg.astype(np.int64) @ G.astype(np.int64)) & 1)  # Eq. 3
        assert np.array_equal(cw[:, s.info], msg)


def test_encoded_words_zero_syndrome_in_oracle(oracle_lib):
    wd = workloads.words("c1", 1, 0, 2.0, 0, 300, fp32=False)
    code = workloads.code("c1")
    assert np.all(oracle_lib.syndrome_ok(code, wd.cw) == 1)
    bad = wd.cw.copy()
    bad[:, 5] ^= 1
    assert not np.any(oracle_lib.syndrome_ok(code, bad))


def test_channel_llr_statistics():
    rng = np.random.default_rng(11)
    s2 = channel.sigma2(2.0, 0.5)
    assert s2 == pytest.approx(1.0 / (10 ** 0.2))
    cw = np.zeros((2000, 500), dtype=np.uint8)
    llr = channel.awgn_llr(cw, s2, rng)
    # consistency of the BI-AWGN LLR: mean 2/sigma^2, variance 4/sigma^2 (= 2 |mean|)
    assert llr.mean() == pytest.approx(2 / s2, rel=5e-3)
    assert llr.var() == pytest.approx(4 / s2, rel=5e-3)
    ones = channel.noiseless_llr(np.ones((1, 4), dtype=np.uint8), s2)
    assert np.all(ones < 0)  # bit 1 -> x = -1 -> negative LLR


def test_blocks_regenerate_independently():
    a = workloads.words("c1", 1, 3, 2.0, 0, 3000, fp32=True)
    b = workloads.words("c1", 1, 3, 2.0, 2047, 10, fp32=True)
    assert np.array_equal(a.llr[2047:2057], b.llr) and np.array_equal(a.cw[2047:2057], b.cw)
    assert a.llr.dtype == np.float32


@pytest.mark.parametrize("i,dv,design_rate", [(0, 9, 0.25), (1, 6, 0.5), (2, 3, 0.75)])
def test_table1_codes(oracle_lib, i, dv, design_rate):
    """Table I: n = 1032, 12 ones per row, 9 / 6 / 3 per column, design rates 1/4, 1/2, 3/4."""
    name = workloads.PAPER["codes"][i]
    code = workloads.code(name)
    assert (code.n, code.m) == (1032, 1032 * dv // 12)
    assert np.all(code.row_degrees() == 12) and np.all(code.col_degrees() == dv)
    assert 1 - code.m / code.n == design_rate
    s = workloads.systematic(name)
    assert s.k / s.n >= design_rate  # dependent rows only raise the rate
    G = s.generator()
    assert not np.any((code.dense().astype(np.int64) @ G.T.astype(np.int64)) & 1)
    wd = workloads.paper_words(i, 50)
    assert np.all(oracle_lib.syndrome_ok(code, wd.cw) == 1)
