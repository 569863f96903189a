"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only, no GPU): the library's
host-only sources (cluster tree, structured QR sweep of Sec. 4 with its HODLR images, Zolotarev
coefficients) and the oracle's band eigensolver, each built with g++/gcc into a small driver of its
own (tests/sanitize/) and run; any sanitizer report or failed check fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1608_01164_amd", "csrc")
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="4")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out
    assert "runtime error" not in out and "AddressSanitizer" not in out and "LeakSanitizer" not in out, out
    assert r.stdout.strip().endswith("ok"), out


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the HIP headers")
def test_library_host_code_sanitized(tmp_path):
    exe = str(tmp_path / "host_main")
    srcs = [os.path.join(ROOT, "tests", "sanitize", "host_main.cpp"), os.path.join(CSRC, "givens.cpp"),
            os.path.join(CSRC, "zolo.cpp"), os.path.join(CSRC, "tree.cpp")]
    subprocess.run(["g++", "-std=c++17", "-fopenmp", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", *SAN, *srcs,
                    "-o", exe], check=True, capture_output=True, timeout=600)
    _run(exe)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_band_eigensolver_sanitized(tmp_path):
    exe = str(tmp_path / "oracle_main")
    srcs = [os.path.join(ROOT, "tests", "sanitize", "oracle_main.c"), os.path.join(ROOT, "oracle", "eig_band.c")]
    subprocess.run(["gcc", "-std=c11", "-fopenmp", *SAN, *srcs, "-lm", "-o", exe], check=True, capture_output=True,
                   timeout=600)
    _run(exe)
