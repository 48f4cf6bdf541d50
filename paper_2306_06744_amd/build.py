"""Build ``liblt.so`` (the HIP library behind include/lt.h) for gfx950 in-tree.

Every translation unit is compiled by hipcc with packed-FP32 instructions
disabled; the flag kernel's unit is also compiled without floating-point
contraction so its FP64 decisions follow the documented operation order, and
so is the construction unit (point -> finest cell).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "liblt.so")
BUILD = os.path.join(HERE, "_build")

SOURCES = ["lt_tree.hip", "lt_flag.hip", "lt_transfer.hip", "lt_split.hip", "lt_mlp.hip", "lt_cycle.hip",
           "lt_build.hip", "lt_fr.hip"]
NO_CONTRACT = {"lt_flag.hip", "lt_build.hip"}
HEADERS = ["keys.hpp", "scan.hpp", "tree.hpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build failed: " + " ".join(cmd))
    return r


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link liblt.so (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        flags = list(COMMON)
        if src in NO_CONTRACT:
            flags.append("-ffp-contract=off")
        cmd = [HIPCC, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        _run(cmd)
        objs.append(obj)
    tmp = SO + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    _run(cmd)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
