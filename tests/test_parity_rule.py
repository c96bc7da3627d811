"""The parity checker itself, exercised on the CPU with mistakes planted in oracle outputs."""
import numpy as np

from oracle.parity import assert_parity, compare
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
