"""Pins of the FP64 oracle against what the mathematics fixes (no GPU)."""
import numpy as np
import pytest

from synth import codes, gf2, workloads


def _map_check(oracle_lib, code, llr, T):
    G = gf2.systematic(code).generator()
    _, post, _, _ = oracle_lib.decode(code, llr, T, early_stop=False, nthreads=2)
    ref = oracle_lib.bitwise_map(G, llr)
    return np.abs(post - ref).max()


@pytest.mark.parametrize("seed", range(6))
def test_cycle_free_equals_bitwise_map(oracle_lib, seed):
    """On a cycle-free Tanner graph sum-product returns exact bitwise MAP posteriors."""
    rng = np.random.default_rng(100 + seed)
    code = codes.tree_code(int(rng.integers(10, 19)), rng, max_deg=5)
    assert gf2.systematic(code).rank == code.m  # a tree's checks are independent
    llr = rng.uniform(-0.9, 0.9, size=(16, code.n))  # keeps every message inside the +-20 clamp
    assert _map_check(oracle_lib, code, llr, 25) < 1e-9


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6, 7])
def test_single_parity_check_odd_and_even(oracle_lib, d):
    """One check of degree d: one iteration is exact MAP, for odd degrees too (sign convention)."""
    code = codes.from_dense(np.ones((1, d), dtype=np.uint8))
    llr = np.random.default_rng(d).normal(0.5, 2.0, size=(32, d))
    assert _map_check(oracle_lib, code, llr, 1) < 1e-9


def test_repetition_chain_sums_llrs(oracle_lib):
    """Chain of degree-2 checks (repetition code): every posterior is the sum of all LLRs."""
    n = 9
    H = np.zeros((n - 1, n), dtype=np.uint8)
    for i in range(n - 1):
        H[i, i] = H[i, i + 1] = 1
    code = codes.from_dense(H)
    llr = np.random.default_rng(2).uniform(-2, 2, size=(5, n))
    _, post, _, _ = oracle_lib.decode(code, llr, n, early_stop=False)
    assert np.allclose(post, llr.sum(axis=1, keepdims=True), atol=1e-12)


def test_clamp_at_20(oracle_lib):
    """v->c messages saturate at +-20: a degree-2 check passes min(|M|, 20) through."""
    code = codes.from_dense(np.ones((1, 2), dtype=np.uint8))
    llr = np.array([[35.0, -1.0], [-50.0, 3.0], [19.5, 0.25]])
    _, post, _, _ = oracle_lib.decode(code, llr, 1, early_stop=False)
    assert np.allclose(post[:, 1], llr[:, 1] + np.clip(llr[:, 0], -20, 20), atol=1e-9)
    assert np.allclose(post[:, 0], llr[:, 0] + llr[:, 1], atol=1e-9)


def test_noiseless_zero_iterations(oracle_lib):
    code = workloads.code("c1")
    wd = workloads.words("c1", 1, 0, 2.0, 0, 50, fp32=False)
    llr = 2.0 * (1.0 - 2.0 * wd.cw) / wd.sigma2
    hard, post, iters, conv = oracle_lib.decode(code, llr, 20, early_stop=True)
    assert np.all(iters == 0) and np.all(conv == 1)
    assert np.array_equal(hard, wd.cw) and np.array_equal(post, llr)


def test_zero_iterations_returns_channel(oracle_lib):
    code = workloads.code("c1")
    wd = workloads.words("c1", 1, 0, 1.0, 0, 20, fp32=False)
    hard, post, iters, _ = oracle_lib.decode(code, wd.llr, 0, early_stop=False)
    assert np.array_equal(post, wd.llr) and np.all(iters == 0)
    assert np.array_equal(hard, (wd.llr <= 0).astype(np.uint8))


def test_early_stop_is_first_zero_syndrome(oracle_lib):
    """iters with early stop = first t whose decisions satisfy H z^T = 0 in a run without it."""
    code = workloads.code("c1")
    wd = workloads.words("c1", 1, 0, 1.5, 0, 40, fp32=False)
    _, post_es, it_es, _ = oracle_lib.decode(code, wd.llr, 20, early_stop=True)
    first = np.full(40, -1)
    for t in range(0, 21):
        hard_t, post_t, _, conv_t = oracle_lib.decode(code, wd.llr, t, early_stop=False)
        new = (first < 0) & (conv_t == 1)
        first[new] = t
        hit = it_es == t
        assert np.array_equal(post_t[hit], post_es[hit])
    first[first < 0] = 20
    assert np.array_equal(first, it_es)


def test_codeword_sign_flip_symmetry(oracle_lib):
    """Flipping the LLR signs on the support of a codeword flips exactly those decisions."""
    code = workloads.code("c1")
    s = workloads.systematic("c1")
    wd = workloads.words("c1", 1, 0, 1.5, 0, 64, fp32=False)
    c2 = s.encode(np.random.default_rng(9).integers(0, 2, size=(64, s.k), dtype=np.uint8))
    flip = 1.0 - 2.0 * c2
    h1, p1, i1, _ = oracle_lib.decode(code, wd.llr, 20, True)
    h2, p2, i2, _ = oracle_lib.decode(code, wd.llr * flip, 20, True)
    assert np.array_equal(i1, i2)
    assert np.allclose(p2, p1 * flip, rtol=1e-12, atol=1e-12)
    tie = np.abs(p1) < 1e-9
    assert np.array_equal((h2 ^ c2)[~tie], h1[~tie])


def test_decodes_c1_waterfall(oracle_lib):
    """Sanity (not from the paper): (3,6) n=96 at 2 dB decodes most words, BER far below the channel's."""
    code = workloads.code("c1")
    wd = workloads.words("c1", 1, 0, 2.0, 0, 1000, fp32=False)
    hard, _, iters, conv = oracle_lib.decode(code, wd.llr, 20, True)
    raw = np.mean((wd.llr <= 0) != wd.cw)
    ber = np.mean(hard != wd.cw)
    assert ber < raw / 3 and conv.mean() > 0.6 and iters.max() <= 20


def test_unrolled_all_ones_is_plain(oracle_lib):
    code = workloads.code("c1")
    wd = workloads.words("c1", 1, 0, 1.5, 0, 30, fp32=False)
    for T in (0, 1, 5, 12):
        w = np.ones((T, code.nnz))
        post_u = oracle_lib.unrolled(code, wd.llr, w)
        _, post_p, _, _ = oracle_lib.decode(code, wd.llr, T, early_stop=False)
        assert np.array_equal(post_u, post_p)


def test_unrolled_weights_scale_messages(oracle_lib):
    """T=1 on one check: L_v = R_v + w_e E_e, with E from the unweighted channel messages."""
    code = codes.from_dense(np.ones((1, 4), dtype=np.uint8))
    llr = np.array([[0.5, -1.0, 2.0, 1.5]])
    w = np.array([[0.5, 2.0, -1.0, 0.0]])
    ones = oracle_lib.unrolled(code, llr, np.ones_like(w)) - llr
    post = oracle_lib.unrolled(code, llr, w)
    assert np.allclose(post, llr + w[0] * ones[0], atol=1e-12)


def test_reference_gradient_matches_finite_differences(oracle_lib):
    from oracle import grad

    code = workloads.code("c1")
    wd = workloads.words("c1", 1, 0, 2.0, 0, 6, fp32=False)
    T = 4
    w = np.random.default_rng(3).normal(1.0, 0.1, size=(T, code.nnz))
    loss, gl, gw = grad.reference_grad(code, wd.llr, w, wd.cw)
    assert loss == pytest.approx(grad.loss_c(code, wd.llr, w, wd.cw), rel=1e-12)
    rng = np.random.default_rng(4)
    cw_ = [(int(rng.integers(T)), int(rng.integers(code.nnz))) for _ in range(12)]
    cl_ = [(int(rng.integers(6)), int(rng.integers(code.n))) for _ in range(12)]
    fw, fl = grad.fd_grad(code, wd.llr, w, wd.cw, cw_, cl_)
    aw = np.array([gw[t, e] for t, e in cw_])
    al = np.array([gl[b, v] for b, v in cl_])
    scale_w, scale_l = np.abs(gw).max(), np.abs(gl).max()
    assert np.abs(fw - aw).max() <= 1e-6 * scale_w + 1e-10
    assert np.abs(fl - al).max() <= 1e-6 * scale_l + 1e-10


def test_reference_gradient_single_check_closed_form():
    """T=1, one check: dL_v/dlambda_u = 2 * d atanh(prod)/d lambda_u, written from the chain rule."""
    from oracle import grad
    import torch

    d = 4
    code = codes.from_dense(np.ones((1, d), dtype=np.uint8))
    lam = np.array([[0.7, -1.2, 2.5, 0.3]])
    w = np.ones((1, d))
    lt = torch.tensor(lam, requires_grad=True)
    L = grad.forward_torch(code, lt, torch.tensor(w))
    J = np.stack([torch.autograd.grad(L[0, v], lt, retain_graph=True)[0].numpy()[0] for v in range(d)])
    th = np.tanh(lam[0] / 2)
    for v in range(d):
        others = [u for u in range(d) if u != v]
        p = np.prod(th[others])
        for u in range(d):
            if u == v:
                expect = 1.0
            else:
                rest = np.prod(th[[x for x in others if x != u]])
                expect = 2.0 / (1 - p * p) * rest * 0.5 * (1 - th[u] ** 2)
            assert J[v, u] == pytest.approx(expect, rel=1e-10, abs=1e-12)


@pytest.mark.parametrize("which", ["fig1", "irregular"])
def test_syndrome_ok_is_the_codebook(oracle_lib, which):
    """Over every n-bit word of a small code, the words that pass the oracle's syndrome test
    (Eq. 1) are exactly the 2^k codewords m G of the systematic generator (Eqs. 2-3), which the
    oracle builds by row reduction, not by the syndrome."""
    from oracle import encode as OE
    from oracle import map as OM

    if which == "fig1":
        code = codes.fig1_matrix()
    else:
        rng = np.random.default_rng(3)
        H = np.zeros((6, 12), dtype=np.uint8)
        for c in range(6):
            H[c, rng.choice(12, size=int(rng.integers(2, 6)), replace=False)] = 1
        code = codes.from_dense(H, "irregular")
    n = code.n
    allw = ((np.arange(1 << n)[:, None] >> np.arange(n)[None, :]) & 1).astype(np.uint8)
    ok = oracle_lib.syndrome_ok(code, allw)
    form = OE.systematic(code)
    book = OM.codebook(form.G)
    assert int(ok.sum()) == len(book) == 1 << form.k
    assert {tuple(r) for r in allw[ok == 1]} == {tuple(r) for r in book}

