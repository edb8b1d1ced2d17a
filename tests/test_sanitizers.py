"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the oracle (plain C with OpenMP; its arithmetic keeps arrays of tens of KB on
worker-thread stacks at 1024 limbs) through a driver that runs every entry
point, and the C-ABI library's host side (argument checks, the workspace
query, the persistent launch's schedule builder) with the sanitizers on the
host pass only -- the GPU code is compiled as usual and never launched."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(exe, tmp_path):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, cwd=tmp_path, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


def test_oracle_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_driver")
    subprocess.run(["gcc", "-std=gnu11", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined",
                    "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "oracle"),
                    os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "mpref.c"),
                    "-o", exe, "-lm"], check=True, timeout=300)
    assert "oracle driver: ok" in _run(exe, tmp_path)


def test_cabi_host_code_under_sanitizers(tmp_path):
    from paper_1308_1536_amd import build
    exe = str(tmp_path / "abi_driver")
    cmd = [build.hipcc(), "-O1", "-g", "-std=c++17", f"--offload-arch={build.ARCH}",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer",
           "-I", build.INCLUDE, "-I", build.CSRC, *build.SOURCES, os.path.join(HERE, "abi_driver.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, timeout=900, capture_output=True)
    assert "abi driver: ok" in _run(exe, tmp_path)
