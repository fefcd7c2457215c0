"""Build step for libdisthist: compiles the HIP sources for gfx950 with hipcc.

    python -m paper_1808_01478_amd.build

Flags that matter for the results:
  -ffp-contract=off   no implicit fused multiply-add; the binary64 path must
                      follow its documented op sequence exactly
  -fno-fast-math      IEEE semantics (correctly rounded binary64 sqrt)
  -Xclang -target-feature -Xclang -packed-fp32-ops
                      no packed binary32 instructions
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libdisthist.so")
SOURCES = ["dh_api.hip", "dh_kernels.hip", "dh_server.hip", "dh_traj.hip", "dh_noalloc.hip"]
ARCH = os.environ.get("DH_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


# The CPU kernel is host code only: AVX2 + FMA (x86-64-v3, every current
# server CPU) and no errno from sqrt/rint, so the row loop vectorizes; the
# results do not depend on either.
CPU_SOURCES = ["dh_cpu.cpp"]
CPU_FLAGS = ["-x", "c++", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
             "-fno-math-errno", "-mavx2", "-mfma", "-Wall"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libdisthist")


def build(verbose: bool = False) -> str:
    """Compile libdisthist.so in place (always recompiles)."""
    tmp = LIB + f".tmp{os.getpid()}"
    objs = []
    for src in CPU_SOURCES:
        obj = os.path.join(PKG, f".{os.path.splitext(src)[0]}.{os.getpid()}.o")
        rocm_inc = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(hipcc()))),
                                "include")
        _run([hipcc(), *CPU_FLAGS, "-D__HIP_PLATFORM_AMD__", f"-I{rocm_inc}",
              f"-I{INCLUDE}", f"-I{CSRC}", "-c",
              os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    try:
        _run([hipcc(), *HIPCC_FLAGS, f"-I{INCLUDE}", f"-I{CSRC}",
              *[os.path.join(CSRC, s) for s in SOURCES], "-x", "none", *objs, "-o", tmp], verbose)
    finally:
        for obj in objs:
            if os.path.exists(obj):
                os.remove(obj)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
