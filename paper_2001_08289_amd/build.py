"""Builds libscfft.so (HIP, gfx950) in-tree with hipcc.

The kernel instantiations are spread over several translation units (one
per pass family and precision) compiled in parallel, then linked into one
shared library.  Objects go to _build/ at the repository root.
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libscfft.so")
OBJDIR = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # packed fp32 instructions stay disabled for every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]

# (source, object name, extra defines)
UNITS = [("scfft.hip", "scfft", []), ("launch_generic.hip", "generic", [])]
for t in ("float", "double"):
    UNITS.append(("launch_xpass.hip", f"xpass_{t}", [f"-DSCFFT_T={t}"]))
    for k in range(11):
        UNITS.append(("launch_smooth.hip", f"smooth{k}_{t}", [f"-DSCFFT_T={t}", f"-DSCFFT_SMK={k}"]))
    for d in (1, 2, 3):
        UNITS.append(("launch_line.hip", f"line{d}_{t}", [f"-DSCFFT_T={t}", f"-DSCFFT_D={d}"]))


def _compile(unit, verbose):
    src, name, defs = unit
    obj = os.path.join(OBJDIR, name + ".o")
    cmd = [HIPCC, *FLAGS, *defs, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(len(UNITS), os.cpu_count() or 4, 16)
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, verbose), UNITS))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
