"""Builds ``libfpde.so`` (HIP sources in ``csrc/``) for gfx950 with hipcc.

Usage: ``python -m paper_1811_03339_amd.build``.  Each source is compiled
to an object file in ``_build/`` (in parallel), then the objects are linked
into the library, which is placed next to this file and loaded by the
package's ctypes binding.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

HERE = Path(__file__).resolve().parent
ROOT = HERE.parent
CSRC = HERE / "csrc"
OBJ = HERE / "_build"
LIB = HERE / "libfpde.so"
SOURCES = ["mesh.hip", "walk.hip", "template.hip", "assemble.hip", "tubes.hip", "solve.hip", "lu.hip",
           "divform.hip", "sparse.hip", "forms.hip", "plane.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # the walk's element ids must be reproducible bit for bit: no FMA
    # contraction anywhere; kernels that want FMA call fma() explicitly
    "-ffp-contract=off",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-Wno-unused-result",
]


def _jobs() -> int:
    return max(1, min(16, len(SOURCES), os.cpu_count() or 1))


def build(verbose: bool = False) -> Path:
    OBJ.mkdir(exist_ok=True)
    inc = [f"-I{ROOT / 'include'}", f"-I{CSRC}"]
    srcs = [s for s in SOURCES if (CSRC / s).exists()]

    def compile_one(src: str):
        obj = OBJ / (Path(src).stem + ".o")
        cmd = [HIPCC, *FLAGS, *inc, "-c", "-o", str(obj), str(CSRC / src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        return src, obj, r

    with ThreadPoolExecutor(_jobs()) as ex:
        results = list(ex.map(compile_one, srcs))
    failed = [(s, r) for s, _, r in results if r.returncode != 0]
    for s, r in failed:
        sys.stderr.write(f"--- {s}\n{r.stdout}{r.stderr}")
    if failed:
        raise RuntimeError("hipcc failed to build libfpde.so: " + ", ".join(s for s, _ in failed))
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", str(tmp), *[str(o) for _, o, _ in results]]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed to link libfpde.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
