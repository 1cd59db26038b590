"""The CPU oracle under sanitizers: oracle.c with a small driver that calls
every entry point (ordinary, extreme and special inputs, four threads),
built and run with the address and undefined-behaviour sanitizers, then with
the thread sanitizer (the oracle's thread pool shares a work counter).  Any
report fails the test; both builds must print the same results."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "oracle", "sanitize_driver.c")]


def _build_and_run(tmp_path, flags, name):
    exe = str(tmp_path / name)
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", *flags, "-o", exe, *SRC, "-lm", "-lpthread"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_sanitizers(tmp_path):
    out_asan = _build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                                         "-fno-omit-frame-pointer"], "oracle_asan")
    out_tsan = _build_and_run(tmp_path, ["-fsanitize=thread"], "oracle_tsan")
    assert out_asan == out_tsan
    assert out_asan.count("\n") == 9
