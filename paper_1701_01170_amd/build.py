"""Build the package's native parts in-tree.

  * ``libgr.so``      - the gr_* C-ABI library: host runtime (C++) and the
                        traversal kernels (HIP for gfx950), compiled by hipcc;
  * ``graphgen/libgrgen.so`` - the seeded input generators (C, OpenMP, gcc).

Run ``python -m paper_1701_01170_amd.build`` (or ``__graft_entry__.build()``).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")
LIBGR = os.path.join(HERE, "libgr.so")
LIBGRGEN = os.path.join(HERE, "graphgen", "libgrgen.so")
OFFLOAD_ARCH = "gfx950"

# hipcc flags: gfx950 only; packed fp32 instructions are disabled on purpose.
HIP_FLAGS = [
    f"--offload-arch={OFFLOAD_ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build_graphgen(verbose: bool = False) -> str:
    src = os.path.join(HERE, "graphgen", "graphgen.c")
    _run(["gcc", "-O3", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-Wall", src, "-o", LIBGRGEN],
         verbose)
    return LIBGRGEN


def hip_sources() -> list[str]:
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith(".hip") or f.endswith(".cpp"))


def build_libgr(verbose: bool = False, jobs: int = 8) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = hip_sources()
    objs = []
    procs = []
    for s in srcs:
        o = os.path.join(objdir, os.path.basename(s) + ".o")
        objs.append(o)
        lang = ["-x", "hip"]
        cmd = ["hipcc", *lang, *HIP_FLAGS, "-c", s, "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd)))
        if len(procs) >= jobs:
            s0, p0 = procs.pop(0)
            if p0.wait() != 0:
                raise RuntimeError(f"hipcc failed on {s0}")
    for s0, p0 in procs:
        if p0.wait() != 0:
            raise RuntimeError(f"hipcc failed on {s0}")
    tmp = LIBGR + ".tmp"
    _run(["hipcc", f"--offload-arch={OFFLOAD_ARCH}", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIBGR)
    return LIBGR


def build_all(verbose: bool = False) -> None:
    build_graphgen(verbose)
    if os.path.isdir(CSRC) and hip_sources():
        build_libgr(verbose)


if __name__ == "__main__":
    build_all(verbose="-v" in sys.argv)
