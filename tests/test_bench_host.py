"""Host-side contract of bench.py (no GPU): the refusal of runs on several GPUs, the byte model of
the HBM rooflines, and the counter table keyed to the kernel sources and launch shape."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_byte_model_of_the_hbm_forms():
    # (3,6) n=4096: 16 B per edge and 8 B per variable per word-iteration, 9 B per bit of I/O
    n, E = 4096, 12288
    assert bench.bytes_per_word_iteration(n, E) == 16 * E + 8 * n == 229376
    assert bench.bytes_per_word_iteration(n, E) / E == pytest.approx(18.67, abs=0.01)
    assert bench.io_bytes_per_word(n) == 9 * n


def test_alu_model_and_peaks():
    # 2 exp + 2 log + 2 reciprocal-class + 12.5 plain lane-operations per edge-iteration
    assert bench.ALU_OPS_PER_EDGE == pytest.approx(2 + 2 + 2 + 12.5)
    assert bench.VALU_PEAK_TOPS == pytest.approx(256 * 64 * 2.4e9 / 1e12)
    assert bench.HBM_PEAK_GBS == 8000.0


def test_counters_only_for_the_measured_sources_batch_and_shape(tmp_path, monkeypatch):
    for form, c in bench.COUNTERS.items():
        assert bench.counter(form, 1000, "bytes_per_launch") is None  # another batch: not the measured launch
        got = bench.counter(form, 65536, "bytes_per_launch", c.get("shape"))
        assert got in (None, c["bytes_per_launch"])  # None once the kernel sources change
        if c.get("sha1") and c.get("bytes_per_launch"):
            # an edit of any listed source nulls the figure
            src = os.path.join(ROOT, c["sources"][0])
            fake = tmp_path / "src"
            fake.write_bytes(open(src, "rb").read() + b"\n")
            c2 = dict(c, sources=[str(fake)] + c["sources"][1:])
            monkeypatch.setitem(bench.COUNTERS, form, c2)
            assert bench.counter(form, 65536, "bytes_per_launch", c.get("shape")) is None
            monkeypatch.setitem(bench.COUNTERS, form, c)
    c = bench.COUNTERS["batched"]
    if c.get("sha1") and c.get("bytes_per_launch") and c.get("shape"):
        other = dict(c["shape"], waves=(4 if c["shape"].get("waves") != 4 else 8))
        assert bench.counter("batched", 65536, "bytes_per_launch", other) is None  # another launch shape


def test_cpu_model_is_a_name():
    m = bench.cpu_model()
    assert isinstance(m, str) and m
