"""Build libhhlb.so (HIP for gfx950) in-tree with hipcc.

Run as ``python -m paper_1708_03249_amd.build`` or through
``__graft_entry__.build()``.  Cross-compiles without a GPU.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhhlb.so")
ARCH = os.environ.get("HHLB_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off (see the design notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast", "-fno-fast-math",
]


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = True, out: str | None = None, defines=()) -> str:
    """Compile libhhlb.so (or `out`); `defines` are extra -D tuning switches."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build" + ("_" + "_".join(defines) if defines else ""))
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src, extra in (("tables.cpp", []), ("hhlb_api.hip", [])):
        obj = os.path.join(objdir, src + ".o")
        cmd = [hipcc] + HIP_FLAGS + [f"-D{d}" for d in defines] + extra + [
            "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):  # host-only code: plain C++ compiler
            cmd = [os.environ.get("CXX", "g++"), "-O2", "-std=c++17", "-fPIC", "-c",
                   os.path.join(CSRC, src), "-o", obj]
        _run(cmd)
        objs.append(obj)
    target = out or LIB
    tmp = target + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, target)
    return target


if __name__ == "__main__":
    build()
    sys.exit(0)
