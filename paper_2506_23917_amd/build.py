"""Build the gfx950 shared library libhs.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhs.so")
SOURCES = ["hs_kernels.hip", "hs_runtime.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # no fused multiply-add contraction: the flight must round as the plain method does
         # (cell decisions are bit-exact); only the collision stage's sums and rescale, whose
         # rounding decides no integer, ask for contraction locally (fp contract pragmas)
         "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # no loop-invariant hoisting in the code generator: it lifts the FP64 power,
         # exponential and sine polynomials' constants (and lane-derived addresses) out of the
         # tile loops, where they occupy registers for the whole loop and spill
         "-mllvm", "-disable-machine-licm", "-mllvm", "-disable-licm-promotion",
         "-Wno-unused-command-line-argument"]


def build(verbose: bool = False) -> str:
    """Compile every HIP/C++ source into libhs.so (always recompiles)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    if verbose and r.stderr:
        print(r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
