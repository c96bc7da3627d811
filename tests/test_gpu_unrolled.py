"""Differentiable form: unrolled weighted forward and hand-written adjoint vs the FP64 oracle,
the torch FP64 reference gradient and finite differences."""
import numpy as np
import pytest
import torch

from synth import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2201_04265_amd as P

    assert torch.cuda.is_available()
    return P


@pytest.fixture(scope="module")
def c5(P):
    code = W.code("c5")
    g = P.Graph.from_code(code)
    w = W.c5_weights(10)
    return code, g, w


def bce(post, cw):
    sp = torch.nn.functional.softplus
    return (cw * sp(post) + (1.0 - cw) * sp(-post)).mean()


def gpu_grads(P, g, llr, w, cw):
    x = torch.from_numpy(np.ascontiguousarray(llr, dtype=np.float32)).cuda().requires_grad_(True)
    wt = torch.from_numpy(np.ascontiguousarray(w, dtype=np.float32)).cuda().requires_grad_(True)
    post = P.unrolled_decode(g, x, wt)
    loss = bce(post, torch.from_numpy(cw.astype(np.float32)).cuda())
    loss.backward()
    torch.cuda.synchronize()
    return float(loss.detach()), post.detach().cpu().numpy(), x.grad.cpu().numpy(), wt.grad.cpu().numpy()


@pytest.mark.parametrize("name,cfg,T", [("c5", 5, 10), ("c1", 1, 7), ("c3", 3, 4)])
def test_all_ones_weights_equal_plain_bitwise(P, name, cfg, T):
    code = W.code(name)
    g = P.Graph.from_code(code)
    wd = W.words(name, cfg, 0, 2.0, 0, 300, fp32=True)
    x = torch.from_numpy(wd.llr).cuda()
    w = torch.ones((T, code.nnz), dtype=torch.float32, device="cuda")
    post_u = P.unrolled_decode(g, x, w)
    _, post_p, iters = P.decode(g, x, T, early_stop=False)
    torch.cuda.synchronize()
    assert torch.all(iters == T)
    assert torch.equal(post_u, post_p)


def test_forward_matches_oracle(P, c5, oracle_lib):
    code, g, w = c5
    wd = W.words("c5", 5, 0, 2.0, 0, 200, fp32=True)
    post = P.unrolled_decode(g, torch.from_numpy(wd.llr).cuda(), torch.from_numpy(w).cuda()).cpu().numpy()
    ref = oracle_lib.unrolled(code, wd.llr, w.astype(np.float64))
    rel = np.abs(post - ref) / np.maximum(np.abs(ref), 1.0)
    print("max rel", rel.max())
    assert rel.max() <= 1e-4


def test_adjoint_matches_reference_gradient(P, c5):
    from oracle import grad

    code, g, w = c5
    wd = W.words("c5", 5, 0, 2.0, 0, 32, fp32=True)
    loss_g, _, gl, gw = gpu_grads(P, g, wd.llr, w, wd.cw)
    loss_r, rl, rw = grad.reference_grad(code, wd.llr.astype(np.float64), w.astype(np.float64), wd.cw)
    assert loss_g == pytest.approx(loss_r, rel=1e-5)
    for a, r in ((gw, rw), (gl, rl)):
        err = np.linalg.norm(a - r) / np.linalg.norm(r)
        per = np.abs(a - r) / np.maximum(np.abs(r), 1e-3 * np.abs(r).max())
        print("norm rel", err, "per-coord max", per.max())
        assert err <= 1e-3
        assert per.max() <= 1e-3


def test_adjoint_matches_finite_differences(P, c5):
    """Central differences of the FP64 C forward on 16 words: weights and LLRs sampled at
    random, weights whose downstream v->c sums sit beyond the +-20 clamp (gradient through
    them is zero) or just inside it, and the LLRs of the largest magnitude.  Per coordinate
    within 1e-3 of the difference quotient (floor 1e-3 of the largest), 1e-3 in norm."""
    from oracle import grad

    code, g, w = c5
    B = 16
    wd = W.words("c5", 5, 0, 2.0, 0, B, fp32=True)
    llr64, w64 = wd.llr.astype(np.float64), w.astype(np.float64)
    _, _, gl, gw = gpu_grads(P, g, wd.llr, w, wd.cw)
    rng = np.random.default_rng(7)
    T, E = w.shape
    # A^(t+1) before the clamp, per iteration t >= 1: weight w[t][e] enters the sums of the
    # other edges of e's variable (the sums of the variable minus edge e itself)
    pre = []
    grad.forward_torch(code, torch.from_numpy(llr64), torch.from_numpy(w64), pre_clamp=pre)
    edge_var = np.asarray(code.indices, dtype=np.int64)  # variable of each edge (CSR edge order)
    sat = np.zeros((T, E))
    near = np.zeros((T, E))
    for t in range(1, T):
        A = pre[t - 1].numpy()  # [B, E], the sums that w[t-1] feeds
        per_var_sat = np.zeros(code.n)
        per_var_near = np.zeros(code.n)
        np.add.at(per_var_sat, edge_var, (np.abs(A) > 20.5).sum(0))
        np.add.at(per_var_near, edge_var, ((np.abs(A) > 18.0) & (np.abs(A) < 19.9)).sum(0))
        sat[t - 1] = per_var_sat[edge_var]
        near[t - 1] = per_var_near[edge_var]
    coords_w = [(int(rng.integers(T)), int(rng.integers(E))) for _ in range(32)]
    for score in (sat, near):
        top = np.argsort(score.ravel())[::-1][:16]
        assert score.ravel()[top].min() > 0  # such sums exist at 2.0 dB
        coords_w += [(int(i // E), int(i % E)) for i in top]
    coords_l = [(int(rng.integers(B)), int(rng.integers(code.n))) for _ in range(24)]
    big = np.argsort(np.abs(llr64).ravel())[::-1][:16]
    coords_l += [(int(i // code.n), int(i % code.n)) for i in big]
    fw, fl = grad.fd_grad(code, llr64, w64, wd.cw, coords_w, coords_l)
    aw = np.array([gw[t, e] for t, e in coords_w])
    al = np.array([gl[b, v] for b, v in coords_l])
    for a, f in ((aw, fw), (al, fl)):
        err = np.linalg.norm(a - f) / np.linalg.norm(f)
        per = np.abs(a - f) / np.maximum(np.abs(f), 1e-3 * np.abs(f).max())
        print("FD norm rel", err, "per-coord", per.max(), "coords", len(f))
        assert err <= 1e-3
        assert per.max() <= 1e-3


def test_full_size_deterministic(P, c5):
    """Full batch (4096 words, 10 iterations): finite gradients, bitwise repeatable."""
    code, g, w = c5
    wd = W.words("c5", 5, 0, 2.0, 0, 4096, fp32=True)
    a = gpu_grads(P, g, wd.llr, w, wd.cw)
    b = gpu_grads(P, g, wd.llr, w, wd.cw)
    assert np.isfinite(a[3]).all() and np.isfinite(a[2]).all()
    for x, y in zip(a[1:], b[1:]):
        assert np.array_equal(x, y)


def test_zero_iterations(P, c5):
    code, g, _ = c5
    wd = W.words("c5", 5, 0, 2.0, 0, 70, fp32=True)
    x = torch.from_numpy(wd.llr).cuda().requires_grad_(True)
    w = torch.zeros((0, code.nnz), dtype=torch.float32, device="cuda", requires_grad=True)
    post = P.unrolled_decode(g, x, w)
    assert torch.equal(post.detach(), x.detach())
    post.sum().backward()
    assert torch.equal(x.grad, torch.ones_like(x))


def test_adjoint_reference_gradient_tile_form(P):
    """A code too large for the one-word-per-workgroup form runs the 64-word tile kernels:
    their adjoint against the torch FP64 reference as well."""
    from oracle import grad

    code = W.code("c3")
    g = P.Graph.from_code(code)
    rng = np.random.default_rng(31)
    T = 3
    w = rng.normal(1.0, 0.1, size=(T, code.nnz)).astype(np.float32)
    wd = W.words("c3", 3, 0, 1.5, 0, 3, fp32=True)
    loss_g, _, gl, gw = gpu_grads(P, g, wd.llr, w, wd.cw)
    loss_r, rl, rw = grad.reference_grad(code, wd.llr.astype(np.float64), w.astype(np.float64), wd.cw)
    assert loss_g == pytest.approx(loss_r, rel=1e-5)
    for a, r in ((gw, rw), (gl, rl)):
        err = np.linalg.norm(a - r) / np.linalg.norm(r)
        print("tile form norm rel", err)
        assert err <= 1e-3


def test_batch_sizes_across_group_boundaries(P, c5):
    """The one-word-per-workgroup backward groups words by batch size; ragged batches above
    and below the grouping threshold give finite, deterministic gradients that agree with
    the same words decoded alone."""
    code, g, w = c5
    wd = W.words("c5", 5, 1, 2.0, 0, 2051, fp32=True)
    a = gpu_grads(P, g, wd.llr, w[:3], wd.cw)
    b = gpu_grads(P, g, wd.llr, w[:3], wd.cw)
    for x, y in zip(a[1:], b[1:]):
        assert np.array_equal(x, y)
    small = gpu_grads(P, g, wd.llr[:5], w[:3], wd.cw[:5])
    # per-word outputs do not depend on the other words of the batch
    assert np.array_equal(small[1], a[1][:5])
    scale = 5 / 2051  # the loss is a mean over the batch
    assert np.allclose(small[2] * scale, a[2][:5], rtol=1e-5, atol=1e-9)


@pytest.mark.parametrize("seed", range(2))
def test_irregular_code_lds_form(P, seed):
    """Irregular codes (generic-degree kernels) in the one-word-per-workgroup form: all-ones
    weights equal the plain decoder bit for bit, and the adjoint matches the FP64 reference."""
    from oracle import grad
    from synth import codes

    rng = np.random.default_rng(4100 + seed)
    n = int(rng.integers(80, 200))
    m = int(rng.integers(n // 4, n // 2))
    chk, var = [], []
    for c in range(m):
        d = int(rng.integers(2, 14))
        vs = rng.choice(n, size=d, replace=False)
        chk += [c] * d
        var += list(vs)
    code = codes.from_edges(m, n, np.array(chk), np.array(var))
    g = P.Graph.from_code(code)
    T = 5
    llr = rng.normal(1.5, 2.0, size=(37, n)).astype(np.float32)
    x = torch.from_numpy(llr).cuda()
    post_u = P.unrolled_decode(g, x, torch.ones((T, code.nnz), dtype=torch.float32, device="cuda"))
    _, post_p, _ = P.decode(g, x, T, early_stop=False)
    assert torch.equal(post_u, post_p)
    w = rng.normal(1.0, 0.1, size=(T, code.nnz)).astype(np.float32)
    cw = np.zeros((6, n), dtype=np.uint8)
    loss_g, _, gl, gw = gpu_grads(P, g, llr[:6], w, cw)
    loss_r, rl, rw = grad.reference_grad(code, llr[:6].astype(np.float64), w.astype(np.float64), cw)
    assert loss_g == pytest.approx(loss_r, rel=1e-5)
    for a, r in ((gw, rw), (gl, rl)):
        assert np.linalg.norm(a - r) / np.linalg.norm(r) <= 1e-3
