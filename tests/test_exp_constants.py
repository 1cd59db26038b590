"""The polynomial constants of the device FP64 exponentials are the ones the
committed generator (paper_2108_11560_amd/csrc/gen_exp_poly.py, Remez in
50-digit mpmath) produces, and have the relative errors the kernel comments
state (host only)."""

import importlib.util
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2108_11560_amd", "csrc")


def generator():
    sys.dont_write_bytecode = True  # keep csrc free of caches
    spec = importlib.util.spec_from_file_location("gen_exp_poly", os.path.join(CSRC, "gen_exp_poly.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def horner_constants(function):
    """Literals of `double p = c;` and the following `p = fma(p, r, c);` lines
    of a function in bessel_device.hpp, highest degree first."""
    src = open(os.path.join(CSRC, "bessel_device.hpp")).read()
    body = src[src.index(function):]
    body = body[:body.index("\n}\n")]
    first = re.search(r"double p = ([-+0-9.eE]+);", body)
    rest = re.findall(r"p = fma\(p, r, ([-+0-9.eE]+)\);", body)
    return [float(first.group(1))] + [float(c) for c in rest]


def test_set_up_exponential_degree_10():
    # e^r - 1 = r (c1 + c2 r + ... + c10 r^9), c0 = 1 implicit
    c, worst = generator().coefficients(10, 1)
    assert horner_constants("ExpParts exp_parts(double a)") == list(reversed(c[1:]))
    assert c[0] == 1.0
    assert worst <= 3.1e-16


def test_node_exponential_degree_3_on_the_table_interval():
    c, worst = generator().coefficients(3, 256)
    assert horner_constants("double exp_node_f64(double a)") == list(reversed(c))
    assert worst <= 1.8e-14
