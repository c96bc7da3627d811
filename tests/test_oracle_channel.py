"""Pins of the oracle's encoder and channel draws (CPU only).

The Philox generator is checked against numpy's own Philox4x64-10 bit generator,
an independent implementation; the encoder against brute-force codebooks, the
printed example of Fig. 2, closed forms of structured matrices and Eq. 1; the
normals and LLRs against their distributions and exact special cases.
"""
import numpy as np
import pytest
from scipy import stats

from conftest import read_golden
from oracle import channel as OC
from oracle import encode as OE
from synth import codes, gf2, workloads


def _numpy_philox_block(ctr, key):
    # numpy advances its 256-bit counter by one before producing each block
    c = list(ctr)
    assert c[0] >= 1
    c[0] -= 1
    g = np.random.Philox(counter=np.array(c, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    return g.random_raw(4)


def test_mulhilo_against_integers():
    rng = np.random.default_rng(11)
    a = rng.integers(0, 2 ** 63, size=500, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, size=500,
                                                                                          dtype=np.uint64)
    for b in (OC.M0, OC.M1, np.uint64(2 ** 64 - 1), np.uint64(1)):
        hi, lo = OC.mulhilo(a, b)
        for x, h, l in zip(a[:100], hi[:100], lo[:100]):
            p = int(x) * int(b)
            assert int(h) == p >> 64 and int(l) == p & (2 ** 64 - 1)


@pytest.mark.parametrize("ctr,key", [
    ((1, 0, 0, 0), (0, 0)),
    ((7, 3, 0, 0), (220104265, 2)),
    ((2 ** 40 + 5, 17, 9, 2 ** 63), (2 ** 64 - 1, 12345)),
    ((123456789, 0, 2, 0), (42, 1)),
])
def test_philox_against_numpy(ctr, key):
    ours = OC.philox4x64(np.array([ctr], dtype=np.uint64), key)[0]
    ref = _numpy_philox_block(ctr, key)
    assert np.array_equal(ours, ref)


def test_philox_vectorised_rows_independent():
    rng = np.random.default_rng(3)
    ctr = rng.integers(1, 2 ** 62, size=(64, 4), dtype=np.uint64)
    out = OC.philox4x64(ctr, (5, 9))
    for i in (0, 17, 63):
        assert np.array_equal(out[i], _numpy_philox_block(tuple(int(x) for x in ctr[i]), (5, 9)))


def test_messages_layout_and_offsets():
    a = OC.messages(7, 0, 20, 700)
    assert a.shape == (20, 700) and a.dtype == np.uint8 and set(np.unique(a)) <= {0, 1}
    # words are addressed by absolute index, and shorter messages are prefixes
    assert np.array_equal(OC.messages(7, 5, 10, 700), a[5:15])
    assert np.array_equal(OC.messages(7, 0, 20, 300), a[:, :300])
    # bit i of word w is bit (i mod 64) of Philox output (i div 64) mod 4, block i div 256
    x = OC.philox4x64(np.array([[3, 2, 0, 0]], dtype=np.uint64), (7, OC.DOMAIN_MESSAGE))[0]
    for i in (512, 555, 600, 699):
        q = (i // 64) % 4
        assert a[3, i] == (int(x[q]) >> (i % 64)) & 1
    big = OC.messages(1, 0, 200, 1000)
    assert abs(big.mean() - 0.5) < 5 * 0.5 / np.sqrt(big.size)


def test_box_muller_special_cases():
    top = np.array([2 ** 64 - 1], dtype=np.uint64)  # u1 = 1 -> radius 0
    z0, z1 = OC.box_muller(top, np.array([12345 << 11], dtype=np.uint64))
    assert z0[0] == 0.0 and z1[0] == 0.0
    # u2 = 0: all of the radius goes to the cosine branch; u1 = 2^-53 is the smallest
    z0, z1 = OC.box_muller(np.array([0], dtype=np.uint64), np.array([0], dtype=np.uint64))
    assert z0[0] == np.sqrt(2.0 * 53.0 * np.log(2.0)) and z1[0] == 0.0
    # u2 = 1/4 rotates it to the sine branch (cos(pi/2) is one rounding away from 0)
    z0, z1 = OC.box_muller(np.array([0], dtype=np.uint64), np.array([(1 << 51) << 11], dtype=np.uint64))
    assert abs(z0[0]) < 1e-15 and z1[0] == np.sqrt(2.0 * 53.0 * np.log(2.0))


def test_normals_distribution():
    z = OC.normals(2024, 3, 0, 256, 1000)
    assert z.shape == (256, 1000)
    flat = z.ravel()
    assert stats.kstest(flat, "norm").pvalue > 1e-4
    assert abs(flat.mean()) < 5 / np.sqrt(flat.size)
    assert abs(flat.var() - 1.0) < 5 * np.sqrt(2.0 / flat.size)
    # the cosine and sine members of a pair are uncorrelated
    assert abs(np.corrcoef(z[:, 0::4].ravel(), z[:, 1::4].ravel())[0, 1]) < 5 / np.sqrt(z[:, 0::4].size)
    # streams and word offsets address independent, reproducible draws
    assert np.array_equal(OC.normals(2024, 3, 100, 56, 1000), z[100:156])
    assert np.array_equal(OC.normals(2024, 3, 0, 4, 998), z[:4, :998])
    other = OC.normals(2024, 4, 0, 256, 1000).ravel()
    assert abs(np.corrcoef(flat, other)[0, 1]) < 5 / np.sqrt(flat.size)


def test_llr_statistics_and_symmetry():
    s2 = 0.7
    zeros = np.zeros((128, 500), dtype=np.uint8)
    ones = np.ones_like(zeros)
    l0 = OC.awgn_llr(zeros, s2, 9, 1, 0, f64=True)
    l1 = OC.awgn_llr(ones, s2, 9, 1, 0, f64=True)
    # LLR consistency of the BPSK/AWGN channel: mean 2/sigma^2, variance 4/sigma^2
    assert abs(l0.mean() - 2.0 / s2) < 5 * np.sqrt(4.0 / s2 / l0.size)
    assert abs(l0.var() / (4.0 / s2) - 1.0) < 5 * np.sqrt(2.0 / l0.size)
    # same noise, opposite symbol: the two LLRs differ by 4/sigma^2
    assert np.max(np.abs((l0 - l1) - 4.0 / s2)) < 1e-12
    l32 = OC.awgn_llr(zeros, s2, 9, 1, 0)
    assert l32.dtype == np.float32 and np.array_equal(l32, l0.astype(np.float32))


def test_fig1_codebook_by_brute_force():
    code = codes.fig1_matrix()
    form = OE.systematic(code)
    assert form.rank == 3 and form.k == 5
    H = code.dense().astype(int)
    allw = ((np.arange(256)[:, None] >> np.arange(8)[None, :]) & 1).astype(np.uint8)
    nullspace = {tuple(w) for w in allw if not np.any((H @ w) % 2)}
    msgs = ((np.arange(32)[:, None] >> np.arange(5)[None, :]) & 1).astype(np.uint8)
    enc = OE.encode(form, msgs)
    assert {tuple(r) for r in enc} == nullspace and len(nullspace) == 32
    assert np.array_equal(enc[:, form.info], msgs)  # systematic: the message is copied


def test_fig2_example():
    g = read_golden("fig2_encode.txt")
    assert np.array_equal(OE.encode_with_generator(g["m"][0], g["G"])[0], g["p"][0])


def test_identity_parity_part_closed_form():
    # H = [Q | I_m]: the last m columns are pivots and the parity bits are Q m
    rng = np.random.default_rng(5)
    m, k = 24, 40
    Q = rng.integers(0, 2, size=(m, k), dtype=np.uint8)
    H = np.concatenate([Q, np.eye(m, dtype=np.uint8)], axis=1)
    form = OE.systematic(H)
    assert form.rank == m and np.array_equal(np.sort(form.pivots), np.arange(k, k + m))
    assert np.array_equal(form.info, np.arange(k))
    msg = rng.integers(0, 2, size=(10, k), dtype=np.uint8)
    cw = OE.encode(form, msg)
    assert np.array_equal(cw[:, :k], msg)
    assert np.array_equal(cw[:, k:], (msg.astype(int) @ Q.T.astype(int)) % 2)


@pytest.mark.parametrize("name", ["c1", "paper_r14", "c4_2"])
def test_generator_spans_the_null_space(name):
    code = workloads.code(name)
    form = OE.systematic(code)
    H = code.dense().astype(np.int64)
    G = form.G.astype(np.int64)
    assert not np.any((H @ G.T) % 2)  # Eq. 2
    assert np.array_equal(G[:, form.info], np.eye(form.k, dtype=np.int64))  # full rank k
    assert form.rank == gf2.gf2_rank(code.dense()) and form.k == code.n - form.rank
    if name.startswith("paper") or name == "c1":  # dv bands each sum to the all-ones row
        dv = int(code.col_degrees()[0])
        assert form.rank <= code.m - dv + 1
    # the pivot reading picks the same positions as the word generator's encoder
    s = gf2.systematic(code)
    assert np.array_equal(np.sort(s.pivots), np.sort(form.pivots))
    msg = OC.messages(1, 0, 16, form.k)
    assert np.array_equal(OE.encode(form, msg), s.encode(msg))


def test_error_counts():
    cw = np.zeros((3, 6), dtype=np.uint8)
    hard = cw.copy()
    hard[0, [1, 4]] = 1
    hard[2, 5] = 1
    assert np.array_equal(OC.error_counts(hard, cw, np.array([0, 1, 2])), [3, 1, 2])
