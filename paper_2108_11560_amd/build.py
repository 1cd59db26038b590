"""Build libbessel.so (gfx950) in-tree with hipcc.

Run as ``python -m paper_2108_11560_amd.build``; ``__graft_entry__.build()``
calls :func:`build` too.  Every HIP source is compiled for gfx950 only, with
packed FP32 instructions disabled (``-packed-fp32-ops``).  Also builds the
instruction-rate microbenchmark ``_build/valu_rates`` (``microbench/``) and
the plain-C example ``_build/c_abi_demo`` (``examples/``).
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libbessel.so")

SOURCES = ["bessel_kernels.hip", "bessel_mlp.hip", "bessel_gh.hip", "bessel_deriv.hip"]
# stand-alone programs: name -> source (relative to the package)
PROGRAMS = {"valu_rates": os.path.join("microbench", "valu_rates.hip")}
# C programs against the C ABI (plain C, linked to libbessel.so)
C_PROGRAMS = {"c_abi_demo": os.path.join("examples", "c_abi_demo.c")}
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

ARCH = "gfx950"

HIP_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA results in ordinary VGPRs: the network reads every accumulator
    # back on the VALU, which the AGPR form would cost one copy each
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wall",
    "-Wno-unused-command-line-argument",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile every source to an object, then link libbessel.so."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), *HIP_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for name, src in PROGRAMS.items():
        cmd = [hipcc(), *HIP_FLAGS, os.path.join(HERE, src), "-o", os.path.join(objdir, name)]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    for name, src in C_PROGRAMS.items():
        # the HIP runtime header needs its platform macro when read by a C compiler
        cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", INCLUDE,
               "-I", os.path.join(ROCM, "include"), os.path.join(HERE, src), "-o", os.path.join(objdir, name),
               "-L", HERE, "-lbessel", "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lm",
               "-Wl,-rpath,$ORIGIN/.."]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
