"""Pins of the oracle's state-in/state-out decode and of its FP32-storage build (no GPU)."""
import numpy as np
import pytest

from synth import codes, gf2, workloads


def _chain(n):
    H = np.zeros((n - 1, n), dtype=np.uint8)
    for i in range(n - 1):
        H[i, i] = H[i, i + 1] = 1
    return codes.from_dense(H)


@pytest.mark.parametrize("name,snr", [("c1", 1.5), ("c4_3", 1.4)])
def test_resume_equals_continuous_decode(oracle_lib, name, snr):
    """Flooding iterations are a function of the c->v state alone (Algorithm 1): t iterations,
    then u more from the exported state, equal t + u iterations, bit for bit in FP64."""
    code = workloads.code(name)
    wd = workloads.words(name, 9, 0, snr, 0, 40)
    for t, u in ((1, 1), (3, 4), (6, 0)):
        *_, Et = oracle_lib.decode_ex(code, wd.llr, t, False)
        h1, p1, i1, _, E1 = oracle_lib.decode_ex(code, wd.llr, u, False, init_cv=Et)
        h2, p2, i2, _, E2 = oracle_lib.decode_ex(code, wd.llr, t + u, False)
        assert np.array_equal(p1, p2) and np.array_equal(E1, E2) and np.array_equal(h1, h2)


def test_zero_state_equals_plain_decode(oracle_lib):
    code = workloads.code("c1")
    wd = workloads.words("c1", 1, 0, 2.0, 0, 100, fp32=False)
    h, p, i, c = oracle_lib.decode(code, wd.llr, 20, True)
    h2, p2, i2, c2, E = oracle_lib.decode_ex(code, wd.llr, 20, True, init_cv=np.zeros((100, code.nnz)))
    assert np.array_equal(p, p2) and np.array_equal(i, i2) and np.array_equal(h, h2)


def test_degree_two_checks_pass_messages_from_a_state(oracle_lib):
    """Repetition chain (checks of degree 2): 2 atanh(tanh(x/2)) = x, so one iteration from a
    state E^(0) sends each variable's extrinsic sum (clamped to +-20) straight to its
    neighbour: E^(1) on edge (c, w) = clamp(R_v + E^(0) on v's other edge), v the other end."""
    n = 7
    code = _chain(n)
    rng = np.random.default_rng(4)
    llr = rng.uniform(-3, 3, size=(5, n))
    E0 = rng.uniform(-12, 12, size=(5, code.nnz))  # large enough that some sums clamp
    _, post, _, _, E1 = oracle_lib.decode_ex(code, llr, 1, False, init_cv=E0)
    # CSR order: check i has edges 2i (variable i) and 2i + 1 (variable i + 1)
    for b in range(5):
        ext = {}  # (variable, check) -> R_v + sum of E^(0) on v's other checks
        for v in range(n):
            for c in (v - 1, v):
                if 0 <= c < n - 1:
                    other = [cc for cc in (v - 1, v) if 0 <= cc < n - 1 and cc != c]
                    s = llr[b, v] + sum(E0[b, 2 * cc + (1 if cc == v - 1 else 0)] for cc in other)
                    ext[(v, c)] = np.clip(s, -20, 20)
        want = np.zeros(code.nnz)
        for c in range(n - 1):
            want[2 * c] = ext[(c + 1, c)]      # to variable c from variable c + 1
            want[2 * c + 1] = ext[(c, c)]      # to variable c + 1 from variable c
        # tanh/atanh round trip in FP64: ~1e-16 / (1 - tanh^2(x/2)) absolute, 1.4e-8 at |x| = 20
        assert np.allclose(E1[b], want, rtol=0, atol=5e-8)
        Lw = llr[b].copy()
        for c in range(n - 1):
            Lw[c] += want[2 * c]
            Lw[c + 1] += want[2 * c + 1]
        assert np.allclose(post[b], Lw, rtol=0, atol=1e-7)


def test_iteration_zero_uses_the_state(oracle_lib):
    """With early stop, a starting state whose posterior R + sum_c E (Eq. 7) has the signs of
    a codeword stops at iteration 0 and returns that posterior; E returned unchanged."""
    code = workloads.code("c1")
    s = gf2.systematic(code)
    msg = np.random.default_rng(1).integers(0, 2, size=(3, s.k), dtype=np.uint8)
    cw = s.encode(msg)
    x = 1.0 - 2.0 * cw
    llr = -0.3 * x  # channel alone points at the complement: not a codeword in general
    E0 = np.zeros((3, code.nnz))
    E0[:, :] = (x[:, code.indices]) * 0.5  # each variable receives 3 x 0.5 towards its codeword bit
    h, p, i, conv, E = oracle_lib.decode_ex(code, llr, 20, True, init_cv=E0)
    assert np.all(i == 0) and np.all(conv == 1)
    assert np.allclose(p, llr + 1.5 * x, atol=1e-12)
    assert np.array_equal(h, cw) and np.array_equal(E, E0)


@pytest.mark.parametrize("seed", range(3))
def test_store32_build_on_trees_is_map_within_fp32_rounding(oracle_lib, seed):
    """The FP32-storage build rounds what it stores; on a cycle-free graph, where sum-product is
    exact bitwise MAP, its posteriors stay within a few FP32 roundings of MAP and are FP32 values."""
    rng = np.random.default_rng(700 + seed)
    code = codes.tree_code(int(rng.integers(10, 17)), rng, max_deg=5)
    llr = rng.uniform(-0.9, 0.9, size=(8, code.n))
    G = gf2.systematic(code).generator()
    ref = oracle_lib.bitwise_map(G, llr)
    _, p32, _, _, _ = oracle_lib.decode_ex(code, llr, 25, False, store32=True)
    assert np.array_equal(p32, p32.astype(np.float32).astype(np.float64))
    err = np.abs(p32 - ref) / np.maximum(np.abs(ref), 1.0)
    assert err.max() < 2e-6
    _, p64, _, _, _ = oracle_lib.decode_ex(code, llr, 25, False)
    assert np.abs(p64 - ref).max() < 1e-9  # the FP64 build of the same source is exact MAP here
