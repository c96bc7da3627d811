"""The parity checker itself, exercised on the CPU with mistakes planted in oracle outputs."""
import numpy as np
import pytest

from oracle.parity import FACTOR, REL, assert_parity, compare
from synth import workloads


def _ref(oracle_lib, B=64):
    code = workloads.code("c1")
    wd = workloads.words("c1", 1, 0, 2.5, 0, B, fp32=True)
    return code, wd, oracle_lib.decode(code, wd.llr, 20, True)


def test_identical_outputs_pass(oracle_lib):
    code, wd, (h, p, i, _) = _ref(oracle_lib)
    st = compare(h, p, i, h.copy(), p.astype(np.float32), i.copy(), oracle_lib, code, wd.llr, 20)
    assert_parity(st)


def test_planted_posterior_error_is_caught(oracle_lib):
    code, wd, (h, p, i, _) = _ref(oracle_lib)
    w = int(np.argmin(i))  # an early-stopping, well-conditioned word
    bad = p.copy()
    bad[w, 3] *= 1.0 + 5e-3
    st = compare(h, p, i, h, bad, i, oracle_lib, code, wd.llr, 20)
    assert st["bad_post_words"] == [w]


def test_planted_decision_and_iteration_errors_are_caught(oracle_lib):
    code, wd, (h, p, i, _) = _ref(oracle_lib)
    hb = h.copy()
    big = np.argmax(np.abs(p[5]))
    hb[5, big] ^= 1
    ib = i.copy()
    ib[7] += 1
    st = compare(h, p, i, hb, p, ib, oracle_lib, code, wd.llr, 20)
    assert st["mismatched_words"] == 2


def test_non_tie_flip_is_caught_even_beside_a_tie(oracle_lib):
    """A word with a tie bit elsewhere gets no excuse for a flipped decision on a clear bit."""
    code, wd, (h, p, i, _) = _ref(oracle_lib)
    w = 9
    gp = p.copy()
    tie_v = int(np.argmin(np.abs(p[w])))
    gp[w, tie_v] = 1e-4  # a tie on the GPU side at another bit
    hb = h.copy()
    clear = int(np.argmax(np.abs(p[w])))
    hb[w, clear] ^= 1
    st = compare(h, p, i, hb, gp, i, oracle_lib, code, wd.llr, 20)
    assert st["mismatched_words"] == 1 and st["tie_exceptions"] == 0
    # the same flip on the tie bit itself is an excused tie
    hb2 = h.copy()
    hb2[w, tie_v] ^= 1
    gp2 = p.copy()
    gp2[w, tie_v] = -np.sign(p[w, tie_v]) * 1e-4 if p[w, tie_v] != 0 else 1e-4
    p2 = p.copy()
    p2[w, tie_v] = np.sign(p[w, tie_v]) * 5e-4
    st2 = compare(h, p2, i, hb2, gp2, i, oracle_lib, code, wd.llr, 20)
    assert st2["mismatched_words"] == 0 and st2["tie_exceptions"] == 1


def _ill_conditioned(oracle_lib):
    """A word of the C1 code on which correctly rounded FP32 storage alone moves the posterior
    past REL / FACTOR (found by the FP32-storage oracle, 4000 words at 2.5 dB)."""
    code = workloads.code("c1")
    wd = workloads.words("c1", 1, 7, 2.5, 0, 4000, fp32=False)
    h, p, i, _ = oracle_lib.decode(code, wd.llr, 20, True)
    _, p32, i32, _, _ = oracle_lib.decode_ex(code, wd.llr, 20, True, store32=True)
    dev = (np.abs(p32 - p) / np.maximum(np.abs(p), 1)).max(axis=1)
    dev[i32 != i] = 0
    w = int(np.argmax(dev))
    assert dev[w] > REL / FACTOR
    sl = slice(w, w + 1)
    return code, wd.llr[sl], h[sl], p[sl], i[sl]


def test_fp32_ill_conditioned_word_is_bounded_not_waived(oracle_lib):
    """An error within FACTOR times the FP32-storage oracle's own deviation on an
    ill-conditioned word is excused; a planted error far beyond it is caught."""
    code, llr, h, p, i = _ill_conditioned(oracle_lib)
    _, p32, _, _, _ = oracle_lib.decode_ex(code, llr, 20, True, store32=True)
    st = compare(h, p, i, h, p32, i, oracle_lib, code, llr, 20)
    assert st["words_over_1e4"] in (0, 1) and not st["bad_post_words"]
    s32 = st["fp32_sensitivity"].get(0, REL)
    v = int(np.argmax(np.abs(p32 - p)))
    bad = p.copy()
    bad[0, v] += 3 * FACTOR * s32 * max(abs(p[0, v]), 1.0)
    st = compare(h, p, i, h, bad, i, oracle_lib, code, llr, 20)
    assert st["bad_post_words"] == [0], st


def test_iteration_mismatch_without_tie_is_caught(oracle_lib):
    """An iteration count that differs where the oracle's posterior at the deciding iteration
    has no tie bit is a mismatch, whatever ties the final posteriors hold."""
    code, wd, (h, p, i, _) = _ref(oracle_lib)
    w = int(np.flatnonzero(i >= 2)[0])
    _, pt, _, _ = oracle_lib.decode(code, wd.llr[w:w + 1], int(i[w]) - 1, False)
    assert np.abs(pt).min() >= 1e-3
    ib = i.copy()
    ib[w] -= 1
    gp = p.copy()
    gp[w, 0] = 1e-5  # a tie in the final posterior does not excuse it
    st = compare(h, p, i, h, gp, ib, oracle_lib, code, wd.llr, 20)
    assert st["mismatched_words"] == 1
