"""Compile libmt.so for gfx950 with hipcc (in-tree, no JIT cache)."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "mt.hip")
INC = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libmt.so")
# measurement kernels (ceilings the benchmark reports beside the path)
MICRO_SRC = os.path.join(PKG, "csrc", "micro.hip")
MICRO_LIB = os.path.join(PKG, "libmt_micro.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed fp32 instructions stay off (device code only; the host pass warns)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-Wall",
    "-Wno-unused-function",
]


def _compile(src: str, out: str, verbose: bool):
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", INC, "-o", tmp, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """Compile both libraries every time it is called; returns the path of
    the merge-tree library."""
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(2) as ex:
        jobs = [ex.submit(_compile, SRC, LIB, verbose), ex.submit(_compile, MICRO_SRC, MICRO_LIB, verbose)]
        for j in jobs:
            j.result()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
