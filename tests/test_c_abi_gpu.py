"""The C ABI used from plain C with no Python in the loop: the example
program (examples/c_abi_demo.c, built with the library) runs as a child
process and checks log K_{1/2}, its first and second x-derivatives and the
second x-derivative of K itself (bessel_logdk) against the closed form
(DLMF 10.39.2), and the error path of an invalid nbins."""

import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_2108_11560_amd", "_build", "c_abi_demo")


def test_c_program():
    if not os.path.exists(EXE):
        pytest.fail("c_abi_demo is not built (python -m paper_2108_11560_amd.build)")
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.count(" ok ") == 5
