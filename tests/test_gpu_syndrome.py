"""ldpc_syndrome (the syndrome test of Eq. 1 on given decisions) against the oracle's, bit for bit:
decoder outputs with satisfied and unsatisfied words, codewords and single flips, bytes other than
0/1 (nonzero = 1), a batch longer than one launch's workgroups, a word longer than the LDS-staged
size, and the decoders' own stopping rule."""
import numpy as np
import pytest
import torch

from synth import codes, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2201_04265_amd as P

    assert torch.cuda.is_available()
    return P


def _gpu_ok(P, g, words):
    ok = P.syndrome_ok(g, torch.from_numpy(np.ascontiguousarray(words, dtype=np.uint8)).cuda())
    torch.cuda.synchronize()
    return ok.cpu().numpy()


def _flips(cw, rng):
    """Codewords, and codewords with one, two or three positions flipped."""
    out = [cw]
    for nflip in (1, 2, 3):
        w = cw.copy()
        for b in range(w.shape[0]):
            w[b, rng.choice(w.shape[1], size=nflip, replace=False)] ^= 1
        out.append(w)
    return np.concatenate(out)


@pytest.mark.parametrize("name,cfg,ebn0,B,T", [("c1", 1, 1.0, 1000, 3), ("c2", 2, 2.0, 300, 10),
                                               ("c3", 3, 3.0, 70, 8), ("c4_1", 4, 2.25, 130, 8),
                                               ("c4_5", 4, 3.0, 200, 10)])
def test_equals_oracle_on_decoder_outputs(P, oracle_lib, name, cfg, ebn0, B, T):
    """Hard decisions after a few iterations without early stop (some words satisfy every check,
    some do not), the transmitted codewords, and codewords with 1-3 flips."""
    code = workloads.code(name)
    g = P.Graph.from_code(code)
    key = int(name[3:]) if name.startswith("c4_") else None
    wd = workloads.words(name, cfg, 0, ebn0, 0, B, fp32=True, **({"code_key": key} if key is not None else {}))
    hard, _, _ = P.decode(g, torch.from_numpy(wd.llr).cuda(), T, False)
    words = np.concatenate([hard.cpu().numpy(), _flips(wd.cw, np.random.default_rng(B))])
    ref = oracle_lib.syndrome_ok(code, words)
    got = _gpu_ok(P, g, words)
    n_ok = int(ref[:B].sum())
    print(name, "decoded words passing", n_ok, "of", B)
    assert 0 < n_ok < B  # both outcomes occur among the decoder outputs
    assert np.array_equal(got, ref)
    assert np.all(got[B:2 * B] == 1) and not np.any(got[2 * B:3 * B])


def test_nonzero_bytes_are_ones(P, oracle_lib):
    code = workloads.code("c1")
    g = P.Graph.from_code(code)
    wd = workloads.words("c1", 1, 0, 2.0, 0, 400, fp32=True)
    rng = np.random.default_rng(11)
    words = _flips(wd.cw, rng)
    scaled = words * rng.integers(1, 256, size=words.shape).astype(np.uint8)  # 1 -> any nonzero byte
    got = _gpu_ok(P, g, scaled)
    assert np.array_equal(got, oracle_lib.syndrome_ok(code, (scaled != 0).astype(np.uint8)))
    assert np.array_equal(got, _gpu_ok(P, g, words))


def test_batch_beyond_one_launch_ragged(P, oracle_lib):
    """More words than one launch has workgroups (8192), in a ragged count."""
    code = workloads.code("c1")
    g = P.Graph.from_code(code)
    B = 9001
    wd = workloads.words("c1", 1, 0, 1.5, 0, B, fp32=True)
    hard, _, _ = P.decode(g, torch.from_numpy(wd.llr).cuda(), 2, False)
    words = hard.cpu().numpy()
    ref = oracle_lib.syndrome_ok(code, words)
    assert 0 < int(ref.sum()) < B
    assert np.array_equal(_gpu_ok(P, g, words), ref)
    assert np.array_equal(_gpu_ok(P, g, words[:1]), ref[:1])


def test_word_longer_than_the_staged_size(P, oracle_lib):
    """n = 70002 > 65536: the checks gather from global memory instead of LDS."""
    code = codes.gallager_band(70002, 3, 6, np.random.default_rng(5), "band(3,6)n70002")
    g = P.Graph.from_code(code)
    rng = np.random.default_rng(6)
    words = _flips(np.zeros((6, code.n), dtype=np.uint8), rng)
    words[0, :] = 1  # all ones: every check of even degree is satisfied
    ref = oracle_lib.syndrome_ok(code, words)
    assert ref[0] == 1 and np.all(ref[1:6] == 1) and not np.any(ref[6:12])
    assert np.array_equal(_gpu_ok(P, g, words), ref)


def test_agrees_with_the_decoders_stopping_rule(P):
    """With early stop, a word that stopped before the limit satisfies every check, and among the
    words at the limit the test finds those that do not; the stream form's decisions (bitwise equal
    to the plain decoder's) give the same results."""
    code = workloads.code("c2")
    g = P.Graph.from_code(code)
    wd = workloads.words("c2", 2, 0, 1.5, 0, 2000, fp32=True)
    x = torch.from_numpy(wd.llr).cuda()
    T = 12
    hard, _, iters = P.decode(g, x, T, True)
    ok = P.syndrome_ok(g, hard).cpu().numpy()
    it = iters.cpu().numpy()
    assert np.all(ok[it < T] == 1)
    assert np.any(it == T) and np.any(ok[it == T] == 0)
    hs, _, _ = P.decode_stream(g, x, T, True)
    assert np.array_equal(P.syndrome_ok(g, hs).cpu().numpy(), ok)


def test_empty_batch_and_bad_shape(P):
    code = workloads.code("c1")
    g = P.Graph.from_code(code)
    assert P.syndrome_ok(g, torch.zeros((0, code.n), dtype=torch.uint8, device="cuda")).shape == (0,)
    with pytest.raises(ValueError):
        P.syndrome_ok(g, torch.zeros((3, code.n + 1), dtype=torch.uint8, device="cuda"))
