"""Host-side contract of bench.py (no GPU): the refusal of runs on several GPUs, the byte model of
the HBM rooflines, and the counter-traffic table keyed to the kernel sources."""
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


def test_valu_model_and_peaks():
    assert bench.STREAM_VALU_SLOTS_PER_EDGE == pytest.approx(89 / 6 + 67 / 9)
    assert bench.VALU_PEAK_TOPS == pytest.approx(256 * 64 * 2.4e9 / 1e12)
    assert bench.HBM_PEAK_GBS == 8000.0


def test_counter_traffic_only_for_the_measured_sources_and_batch():
    for form in ("stream", "batched"):
        c = bench.COUNTER_TRAFFIC[form]
        assert c["bytes_per_launch"] == c["read_bytes"] + c["write_bytes"]
        assert bench.counter_traffic(form, 1000) is None  # another batch: not the measured launch
        got = bench.counter_traffic(form, 65536)
        assert got in (None, c["bytes_per_launch"])  # None once the kernel sources change
    assert bench.counter_traffic("plain", 65536) is None


def test_cpu_model_is_a_name():
    m = bench.cpu_model()
    assert isinstance(m, str) and m
