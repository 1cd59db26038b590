"""The library's host code under the address and undefined-behaviour
sanitizers (CPU): every source is rebuilt with the build's flags plus
host-only sanitizer flags (the device code is unchanged), linked into a
separate library, and a C driver (tests/abi_errors_driver.c) runs every
entry point's argument checks, statuses and messages, the batch-size policy
and the version string against it.  No GPU is touched: each call returns
from its host-side checks."""

import os
import subprocess

import pytest

from paper_2108_11560_amd import build as B

SAN = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def test_host_code_under_sanitizers(tmp_path):
    try:
        hipcc = B.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not found")
    objs = []
    for src in B.SOURCES:
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        subprocess.run([hipcc, *B.HIP_FLAGS, *SAN, "-I", B.INCLUDE, "-I", B.CSRC, "-c",
                        os.path.join(B.CSRC, src), "-o", obj], check=True, capture_output=True)
        objs.append(obj)
    lib = str(tmp_path / "libbessel_san.so")
    subprocess.run([hipcc, f"--offload-arch={B.ARCH}", "-shared", "-fPIC", *SAN, "-o", lib, *objs], check=True,
                   capture_output=True)
    clang = os.path.join(B.ROCM, "llvm", "bin", "clang")
    exe = str(tmp_path / "abi_errors")
    subprocess.run([clang, "-std=c11", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-D__HIP_PLATFORM_AMD__", "-I", B.INCLUDE, "-I", os.path.join(B.ROCM, "include"),
                    os.path.join(os.path.dirname(__file__), "abi_errors_driver.c"), "-o", exe,
                    f"-L{tmp_path}", "-lbessel_san", "-L", os.path.join(B.ROCM, "lib"), "-lamdhip64",
                    f"-Wl,-rpath,{tmp_path}", "-Wl,-rpath," + os.path.join(B.ROCM, "lib")], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr
