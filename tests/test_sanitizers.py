"""Host code and the oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

Two small C/C++ drivers (``tests/sanitize/``) call every entry point of the
CPU oracle and the library's host-side operator construction on small and
degenerate inputs; they are built with ``-fsanitize=address,undefined
-fno-sanitize-recover=all`` and must run clean (any report aborts the
driver).  The oracle and the library stay in separate executables: they
share no code.  GPU code is not built here (no device sanitizers on this
target); these cover the CPU side only.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(cmd_build, exe, tmp_path):
    r = subprocess.run(cmd_build, capture_output=True, text=True, cwd=ROOT)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-2000:]
    # verify_asan_link_order=0: a library preloaded by the environment may come first
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.returncode, r.stdout[-500:], r.stderr[-4000:])


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_sanitized(tmp_path):
    exe = tmp_path / "oracle_drive"
    cmd = ["gcc", "-std=gnu99", "-fopenmp", "-ffp-contract=off", "-fcx-limited-range", *SAN,
           "tests/sanitize/oracle_drive.c", "oracle/fmm_oracle.c", "oracle/mlp_oracle.c", "-o", str(exe), "-lm"]
    _run(cmd, exe, tmp_path)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
def test_host_ops_sanitized(tmp_path):
    exe = tmp_path / "host_drive"
    cmd = ["g++", "-std=c++17", *SAN, "-Ipaper_1108_5815_amd/csrc", "tests/sanitize/host_drive.cpp",
           "paper_1108_5815_amd/csrc/host_ops.cpp", "-o", str(exe)]
    _run(cmd, exe, tmp_path)
