"""Sanitizer runs.

CPU: the oracle (double and complex-step builds) compiled with gcc's
AddressSanitizer and UndefinedBehaviorSanitizer (leak check on) and driven
through every entry point by tests/sanitize/oracle_check.c.

GPU: the library's host code compiled with the same two sanitizers (device
code unchanged) and driven through the C ABI by tests/sanitize/host_check.cpp
(built by tests/sanitize/build_host_check.py, which __graft_entry__.build()
calls).  The HIP runtime allocates for the life of the process, so the leak
check is off there.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = os.path.join(HERE, "sanitize")
ORACLE = os.path.join(ROOT, "oracle")


def _assert_clean(p, last_line):
    out = p.stdout + p.stderr
    assert p.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert last_line in p.stdout, out[-4000:]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_check")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-fopenmp",
           "-ffp-contract=off", "-I", ORACLE, os.path.join(SAN, "oracle_check.c"),
           os.path.join(ORACLE, "hsgn_oracle.c"), os.path.join(ORACLE, "hsgn_oracle_cs.c"),
           "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    p = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    _assert_clean(p, "all cases ran")


def _host_check_state():
    from paper_2510_07539_amd import build as B
    exe = os.path.join(SAN, "host_check")
    if not os.path.exists(exe):
        return exe, "not built"
    t = os.path.getmtime(exe)
    deps = B.DEPS + [os.path.join(SAN, "host_check.cpp")]
    if any(os.path.getmtime(d) > t for d in deps):
        return exe, "older than its sources"
    return exe, None


@pytest.mark.gpu
def test_library_host_code_asan_ubsan():
    exe, why = _host_check_state()
    if why:
        pytest.skip("tests/sanitize/host_check is %s: run __graft_entry__.build()" % why)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    print("running", exe, flush=True)
    p = subprocess.run([exe], capture_output=True, text=True, timeout=100, env=env)
    print(p.stdout[-3000:], flush=True)
    _assert_clean(p, "all calls returned as expected")
