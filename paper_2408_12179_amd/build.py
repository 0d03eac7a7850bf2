"""Build the HIP library ``libhprlp.so`` for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build", "hprlp")
LIB = os.path.join(PKG, "libhprlp.so")
EXAMPLE = os.path.join(PKG, "examples", "solve_transport")
SOURCES = ["kernels.hip", "prep.hip", "t1zero.hip", "setup.cpp", "api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("HPRLP_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS]
    if src.endswith(".cpp"):
        cmd += ["-x", "hip"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = False) -> str:
    """Compile every source and link the shared library; always rebuilds."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    subprocess.run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs], check=True)
    os.replace(tmp, LIB)
    # the C example: plain C against the C ABI and the HIP runtime API only
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-D__HIP_PLATFORM_AMD__",
                    "-I", os.path.join(rocm, "include"), "-I", os.path.join(ROOT, "include"),
                    EXAMPLE + ".c", "-L", PKG, "-lhprlp", "-L", os.path.join(rocm, "lib"),
                    "-lamdhip64", "-lm", "-Wl,-rpath,$ORIGIN/..",
                    "-Wl,-rpath," + os.path.join(rocm, "lib"), "-o", EXAMPLE], check=True)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
