"""Compile the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc, IEEE double arithmetic (no fast-math), OpenMP for independent
rays / key points.

`python -m oracle.build --sanitize` builds oracle/liboracle.asan.so instead:
the same source under AddressSanitizer and UndefinedBehaviorSanitizer, with
ROCm's clang so that it shares one sanitizer runtime with the sanitized host
code of librte (see paper_1809_06417_amd/build.py). The loader takes it when
RTE_SANITIZE=1 is set; run with that runtime preloaded (LD_PRELOAD of
ASAN_RUNTIME below, ASAN_OPTIONS=detect_leaks=0).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rte_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
SAN_LIB = os.path.join(HERE, "liboracle.asan.so")
CLANG = "/opt/rocm/llvm/bin/clang"


def asan_runtime() -> str:
    """Path of clang's shared AddressSanitizer runtime (to preload)."""
    out = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                         text=True, check=True).stdout.strip()
    if not os.path.isabs(out):
        import glob
        hits = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        out = hits[0] if hits else out
    return out


def build(verbose: bool = False, sanitize: bool = False) -> str:
    if sanitize:
        cmd = [CLANG, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fno-fast-math", "-ffp-contract=off",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-shared-libsan", "-fopenmp",
               "-fPIC", "-shared", "-D_DEFAULT_SOURCE", "-Wall", "-Wextra", "-Wno-unused-parameter",
               "-Wl,-rpath,/opt/rocm/llvm/lib", "-o", SAN_LIB + ".tmp", SRC, "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(SAN_LIB + ".tmp", SAN_LIB)
        return SAN_LIB
    cmd = ["gcc", "-std=c11", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
           "-shared", "-D_DEFAULT_SOURCE", "-Wall", "-Wextra", "-Wno-unused-parameter", "-o",
           LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        build(verbose=True, sanitize=True)
        print("preload:", asan_runtime())
    else:
        build(verbose=True)
    sys.exit(0)
