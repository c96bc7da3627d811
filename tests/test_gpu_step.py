"""One-step ("teacher-forced") parity of Eqs. 5-7 through ldpc_decode_ex.

For each workload, the FP64 oracle decodes sampled words for t iterations without early
stop and returns its c->v state E^(t); that state is rounded to FP32 and both sides run
exactly one flooding iteration from it (Algorithm 1: Eq. 6 from E^(t), Eq. 5, Eq. 7).
Every posterior and every c->v message of the GPU must sit within
1e-4 * max(|x_64|, 1) of the oracle's FP64 value computed from the same rounded state:
no exemption.  This pins the FP32 per-iteration arithmetic independently of how a long
trajectory amplifies rounding.  Hard decisions must agree except on bits with
|L| < 1e-3 (ties, Eq. 8 at L = 0).
"""
import numpy as np
import pytest
import torch

from synth import workloads

pytestmark = pytest.mark.gpu

REL = 1e-4
TIE = 1e-3


@pytest.fixture(scope="module")
def P():
    import paper_2201_04265_amd as P

    assert torch.cuda.is_available()
    return P


def _rel(a, b):
    return np.abs(np.asarray(a, np.float64) - b) / np.maximum(np.abs(b), 1.0)


def one_step(P, oracle_lib, code, llr, ts, label):
    """States after t oracle iterations (t in ts), rounded to FP32; one iteration on each side."""
    g = P.Graph.from_code(code)
    states, rows = [], []
    for t in ts:
        *_, Et = oracle_lib.decode_ex(code, llr, t, False)
        states.append(Et.astype(np.float32))
        rows.append(llr)
    S = np.concatenate(states)
    X = np.concatenate(rows)
    oh, op, oi, _, oE = oracle_lib.decode_ex(code, X, 1, False, init_cv=S.astype(np.float64))
    x = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    gh, gp, gi, gE = P.decode_ex(g, x, 1, False, init_cv=torch.from_numpy(S).cuda())
    torch.cuda.synchronize()
    gh, gp, gi, gE = gh.cpu().numpy(), gp.cpu().numpy(), gi.cpu().numpy(), gE.cpu().numpy()
    assert np.all(gi == 1) and np.all(oi == 1)
    rp, rE = _rel(gp, op), _rel(gE, oE)
    # the same step by the FP32-storage oracle: every stored value correctly rounded
    _, sp, _, _, sE = oracle_lib.decode_ex(code, X, 1, False, init_cv=S.astype(np.float64), store32=True)
    ip, iE = _rel(sp, op), _rel(sE, oE)
    k = np.sqrt(np.mean(rE ** 2)) / max(np.sqrt(np.mean(iE ** 2)), 1e-30)
    print(f"P-step {label}: {X.shape[0]} states (t in {list(ts)}), posterior max {rp.max():.2e} "
          f"median {np.median(rp):.2e}; c->v max {rE.max():.2e} median {np.median(rE):.2e}; correctly rounded "
          f"c->v max {iE.max():.2e}, posterior max {ip.max():.2e}; rms ratio of c->v errors {k:.2f}", flush=True)
    assert rp.max() <= REL, (label, rp.max())
    assert rE.max() <= REL, (label, rE.max())
    diff = gh != oh
    ties = (np.abs(op) < TIE) | (np.abs(gp) < TIE)
    assert not np.any(diff & ~ties), label
    return rp.max(), rE.max()


def test_pstep_c1(P, oracle_lib):
    """(3,6) n=96 band, all 1000 words, FP64 LLRs (rounded on the GPU's ingest)."""
    code = workloads.code("c1")
    wd = workloads.words("c1", 1, 0, 2.0, 0, 1000, fp32=False)
    one_step(P, oracle_lib, code, wd.llr, (0, 1, 5, 10, 19), "C1")


@pytest.mark.parametrize("ebn0", workloads.C2["ebn0s"])
def test_pstep_c2(P, oracle_lib, ebn0):
    """(3,6) n=4096, every Eb/N0 point of the sweep, 96 words spread over the batch."""
    code = workloads.code("c2")
    idx = np.linspace(0, 65535, 96).astype(int)
    blocks = {}
    rows = []
    for w in idx:
        b = w // workloads.BLOCK
        if b not in blocks:
            blocks[b] = workloads.words("c2", 2, workloads.C2["ebn0s"].index(ebn0), ebn0, b * workloads.BLOCK,
                                        workloads.BLOCK).llr
        rows.append(blocks[b][w % workloads.BLOCK])
    llr = np.stack(rows)
    one_step(P, oracle_lib, code, llr, (0, 4, 15, 40), f"C2 {ebn0} dB")


def test_pstep_c3(P, oracle_lib):
    """Quasi-cyclic 22x44 Z=256 (n=11264, check degrees to 22), 16 words."""
    code = workloads.code("c3")
    wd = workloads.words("c3", 3, 0, 1.5, 0, 16)
    one_step(P, oracle_lib, code, wd.llr, (0, 8, 29), "C3")


@pytest.mark.parametrize("i", range(6))
def test_pstep_c4(P, oracle_lib, i):
    """Each code of the mixed batch at its own Eb/N0."""
    name = workloads.C4_CODES[i]
    code = workloads.code(name)
    snr = float(workloads.c4_ebn0()[i])
    cnt = 8 if code.n > 8000 else 32
    wd = workloads.words(name, 4, 0, snr, 0, cnt, code_key=i)
    one_step(P, oracle_lib, code, wd.llr, (0, 6, 30), f"C4 {name} {snr} dB")


def test_pstep_c5_code(P, oracle_lib):
    """The differentiable workload's (3,6) n=1024 code at 2.0 dB (plain weights)."""
    code = workloads.code("c5")
    wd = workloads.words("c5", 5, 0, 2.0, 0, 64)
    one_step(P, oracle_lib, code, wd.llr, (0, 3, 9), "C5 code")


def test_state_roundtrip_and_iteration_zero(P, oracle_lib):
    """A state resumed through init_cv continues the decode exactly: t iterations, export,
    then u more from the export equal t + u iterations on the GPU (bitwise), and with early
    stop a word whose starting state already satisfies every check returns at iteration 0
    with the posterior of that state, as the oracle does."""
    code = workloads.code("c1")
    wd = workloads.words("c1", 1, 0, 1.5, 0, 200, fp32=True)
    g = P.Graph.from_code(code)
    x = torch.from_numpy(wd.llr).cuda()
    h1, p1, i1, E1 = P.decode_ex(g, x, 4, False)
    h2, p2, i2, E2 = P.decode_ex(g, x, 3, False, init_cv=E1)
    h3, p3, i3, E3 = P.decode_ex(g, x, 7, False)
    assert torch.equal(p2, p3) and torch.equal(h2, h3) and torch.equal(E2, E3)
    # iteration 0 from a state, early stop on
    Es = E3.cpu().numpy().astype(np.float64)
    oh, op, oi, _, oE = oracle_lib.decode_ex(code, wd.llr, 20, True, init_cv=Es)
    gh, gp, gi, gE = P.decode_ex(g, x, 20, True, init_cv=E3)
    gi = gi.cpu().numpy()
    stopped0 = oi == 0
    assert stopped0.any()
    assert np.array_equal(gi[stopped0], oi[stopped0])
    assert np.array_equal(gE.cpu().numpy()[stopped0], E3.cpu().numpy()[stopped0])
    assert _rel(gp.cpu().numpy()[stopped0], op[stopped0]).max() <= REL
    # no state given: identical to ldpc_decode, and final state zero for words stopping at 0
    hd, pd, idd = P.decode(g, x, 20, True)
    he, pe, ie, Ee = P.decode_ex(g, x, 20, True)
    assert torch.equal(hd, he) and torch.equal(pd, pe) and torch.equal(idd, ie)
    z = (ie == 0)
    assert torch.all(Ee[z] == 0)
