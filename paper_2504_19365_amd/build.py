"""Build steps for the native libraries of this package.

* ``libagilegen.so``: the seeded input generators (gcc, OpenMP).
* ``libagile.so``: the HIP library for gfx950 that exports the C ABI of include/agile.h.

Both are built in-tree, next to their sources, so that they travel with the repository.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
GEN_SO = os.path.join(PKG, "gen", "libagilegen.so")
AGILE_SO = os.path.join(PKG, "libagile.so")
CSRC = os.path.join(PKG, "csrc")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",
    # packed fp32 forms are kept out of the generated code on purpose
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build_gen() -> str:
    src = os.path.join(PKG, "gen", "agile_gen.c")
    _run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", GEN_SO + ".tmp", src,
          "-lm"])
    os.replace(GEN_SO + ".tmp", GEN_SO)
    return GEN_SO


def build_agile() -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    src = os.path.join(CSRC, "agile.hip")
    _run([hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o",
          AGILE_SO + ".tmp", src])
    os.replace(AGILE_SO + ".tmp", AGILE_SO)
    return AGILE_SO


def build_all() -> None:
    build_gen()
    if os.path.exists(os.path.join(CSRC, "agile.hip")):
        build_agile()


if __name__ == "__main__":
    what = sys.argv[1:] or ["all"]
    for w in what:
        {"gen": build_gen, "agile": build_agile, "all": build_all}[w]()
