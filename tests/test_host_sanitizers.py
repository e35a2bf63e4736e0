"""The library's host code (mesh checks, cluster and block trees, Gauss and
Chebyshev rules, the eigen and QR routines of the recompression, the Green
cross approximation's host construction, the H-matrix coarsening,
H-Cholesky factorisation and substitution program) built with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer and run over meshes of
several sizes and leaf sizes and over rejected inputs
(tests/host_asan_driver.cpp).  No device code is built."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2001_05523_amd", "csrc")
HOST_SOURCES = ["host_trees.cpp", "host_linalg.cpp", "gca_host.cpp", "hmatrix.cpp"]


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_code_under_address_and_undefined_behaviour_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "host_asan")
        cmd = (["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
               + [os.path.join(CSRC, f) for f in HOST_SOURCES]
               + [os.path.join(ROOT, "tests", "host_asan_driver.cpp"), "-pthread", "-o", exe])
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        print(r.stdout[-2000:])
        assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-6000:])
        assert "host checks passed" in r.stdout
