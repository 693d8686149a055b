"""Build libhfmm.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1608_02461_amd.build        # or build() from Python

Objects go to ``_build/`` at the repository root; the shared library is
written next to this file.  Every call recompiles every source.
"""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libhfmm.so")

# (source, object name, extra flags): near.hip is built once per precision and
# column-group width so that its kernel instances compile in parallel
SOURCES = [("tree.hip", "tree", []), ("fmm.hip", "fmm", []), ("fmm3.hip", "fmm3", []), ("solver3.hip", "solver3", []), ("solver.hip", "solver", []),
           ("special.cpp", "special", []), ("abi.cpp", "abi", []), ("noalloc.hip", "noalloc", [])] + [
    ("near.hip", f"near_{t}_{nr}", [f"-DNEAR_T={t}", f"-DNEAR_NR={nr}"])
    for t in ("float", "double") for nr in (1, 2, 4)]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
CFLAGS = [
    "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off: hipcc would otherwise form them from
    # ordinary float code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def _compile(entry):
    src, name, extra = entry
    obj = os.path.join(OBJDIR, name + ".o")
    cmd = [HIPCC, *CFLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose=False):
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = min(len(SOURCES), max(1, min(16, os.cpu_count() or 4)))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
