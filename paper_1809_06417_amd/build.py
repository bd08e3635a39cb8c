"""Compile librte.so (HIP for gfx950) in-tree.

`python -m paper_1809_06417_amd.build --sanitize` builds librte.asan.so, whose
host code (argument validation, plan set-up, LUT builder, launch wrappers) is
compiled with AddressSanitizer and UndefinedBehaviorSanitizer; device code is
built as usual. The binding loads it when RTE_SANITIZE=1 is set (CPU test
runs with clang's shared ASan runtime preloaded; see oracle/build.py).

Every source is compiled with hipcc for gfx950 only. Packed-FP32 instruction
selection is disabled (the packed forms are avoided on this target), and
floating-point contraction is off: the kernels write their fused
multiply-adds explicitly, so the render and the back-projection derive
bit-identical sample positions from the same ray table.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "librte.so")
SAN_LIB = os.path.join(PKG, "librte.asan.so")
SOURCES = ["rte_kernels.hip", "rte_api.cpp", "rte_lut.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall",
          "-Wno-unused-command-line-argument", f"-I{INCLUDE}", f"-I{CSRC}"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"command failed: {' '.join(cmd)}")
    return res


# host-side sanitizers only (each flag applies to the host compilation)
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out_dir = os.path.join(BUILD, "asan") if sanitize else BUILD
    os.makedirs(out_dir, exist_ok=True)
    extra = ["-g"] + HOST_SAN if sanitize else []
    objs = []
    for src in SOURCES:
        obj = os.path.join(out_dir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        _run([HIPCC] + COMMON + extra + lang + ["-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    lib = SAN_LIB if sanitize else LIB
    tmp = lib + ".tmp"
    link_san = HOST_SAN[:4] + ["-Xarch_host", "-shared-libsan"] if sanitize else []
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"] + link_san,
         verbose)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv)
