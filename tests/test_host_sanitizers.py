"""The host code under the sanitizers (no GPU): the graph builder and the kernel layouts
(paper_2201_04265_amd/csrc/host_layout.cpp) and the FP64 oracle (oracle/spa.c) are built
with the address and undefined-behaviour sanitizers (the oracle also with the thread
sanitizer, for its worker threads) and driven on seeded random codes by
tests/host/host_checks.cpp and tests/host/oracle_checks.c."""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT

HOST = os.path.join(ROOT, "tests", "host")
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _run(cmd, exe, env=None):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_graph_builder_and_layouts_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "host_checks")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cmd = ["g++", "-std=c++17"] + SAN + ["-D__HIP_PLATFORM_AMD__", f"-I{rocm}/include", f"-I{ROOT}",
                                        os.path.join(HOST, "host_checks.cpp"),
                                        os.path.join(ROOT, "paper_2201_04265_amd", "csrc", "host_layout.cpp"),
                                        "-o", exe]
    assert "host checks ok" in _run(cmd, exe)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("san", ["asan_ubsan", "tsan"])
def test_oracle_under_sanitizers(tmp_path, san):
    exe = str(tmp_path / f"oracle_checks_{san}")
    flags = SAN if san == "asan_ubsan" else ["-O1", "-g", "-fsanitize=thread"]
    cmd = ["gcc", "-std=c11"] + flags + [os.path.join(HOST, "oracle_checks.c"),
                                         os.path.join(ROOT, "oracle", "spa.c"), "-o", exe, "-lm", "-lpthread"]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1")
    assert "oracle checks ok" in _run(cmd, exe, env)
