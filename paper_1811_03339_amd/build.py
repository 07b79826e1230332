"""Builds ``libfpde.so`` (HIP sources in ``csrc/``) for gfx950 with hipcc.

Usage: ``python -m paper_1811_03339_amd.build``.  The library is placed next
to this file and loaded by the package's ctypes binding.
"""
from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

HERE = Path(__file__).resolve().parent
ROOT = HERE.parent
CSRC = HERE / "csrc"
LIB = HERE / "libfpde.so"
SOURCES = ["mesh.hip", "walk.hip", "template.hip", "assemble.hip", "tubes.hip", "solve.hip", "lu.hip",
           "divform.hip", "sparse.hip", "forms.hip", "plane.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # the walk's element ids must be reproducible bit for bit: no FMA
    # contraction anywhere; kernels that want FMA call fma() explicitly
    "-ffp-contract=off",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-Wno-unused-result",
]


def build(verbose: bool = False) -> Path:
    srcs = [str(CSRC / s) for s in SOURCES]
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [HIPCC, *FLAGS, f"-I{ROOT / 'include'}", f"-I{CSRC}", "-o", str(tmp), *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed to build libfpde.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
