"""Build tests/sanitize/_build/solver_lifecycle: the library's sources and
the driver solver_lifecycle.cpp, with AddressSanitizer and
UndefinedBehaviorSanitizer on the host side only (the device code is built
as for libhhlb.so), linked into one executable.  Also writes the driver's
channel list: every 8th of the 4096 channels of the batched workload
(inputs.batch_draws, PCG64 seed 0), 512 channels of uneven Nx and order.

    python tests/sanitize/build_sanitized.py          # build (objects reused while newer than the sources)
    tests/sanitize/_build/solver_lifecycle host tests/sanitize/_build/channels512.txt
    tests/sanitize/_build/solver_lifecycle gpu  tests/sanitize/_build/channels512.txt   # on a GPU

Cross-compiles without a GPU; about a minute on eight cores the first time.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "_build")
OBJ = os.path.join(OUT, "obj")
EXE = os.path.join(OUT, "solver_lifecycle")
CHANNELS = os.path.join(OUT, "channels512.txt")
CLANG = "/opt/rocm/llvm/bin/clang++"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def _host_only(flags):
    out = []
    for f in flags:
        out += ["-Xarch_host", f]
    return out


def _stale(obj, deps):
    return not os.path.exists(obj) or any(os.path.getmtime(d) > os.path.getmtime(obj) for d in deps)


def write_channels():
    sys.path.insert(0, ROOT)
    from paper_1708_03249_amd.inputs import batch_draws
    with open(CHANNELS + ".tmp", "w") as fh:
        for d in batch_draws(4096, 0)[::8]:
            fh.write(f"{d['Q']} {d['Nx']} {d['Kn']!r} {d['g']!r} {d['T_right']!r}\n")
    os.replace(CHANNELS + ".tmp", CHANNELS)


def build(verbose: bool = False) -> str:
    sys.path.insert(0, ROOT)
    from paper_1708_03249_amd import build as B
    os.makedirs(OBJ, exist_ok=True)
    headers = glob.glob(os.path.join(B.CSRC, "*.hpp")) + glob.glob(os.path.join(B.CSRC, "*.h")) + [
        os.path.join(ROOT, "include", "hhlb.h"), os.path.abspath(__file__), os.path.join(B.HERE, "build.py")]
    cmds, objs = [], []
    for src in B.SOURCES:
        path = os.path.join(B.CSRC, src)
        obj = os.path.join(OBJ, src + ".o")
        objs.append(obj)
        if not _stale(obj, [path] + headers):
            continue
        if src.endswith(".cpp"):
            cmds.append([CLANG, "-O2", "-std=c++17", "-fPIC", "-g1"] + SAN + ["-c", path, "-o", obj])
        else:
            cmds.append([HIPCC] + B.HIP_FLAGS + B.SOURCE_FLAGS.get(src, []) + _host_only(SAN + ["-g1"]) +
                        ["-c", path, "-o", obj])
    drv = os.path.join(HERE, "solver_lifecycle.cpp")
    dobj = os.path.join(OBJ, "solver_lifecycle.o")
    objs.append(dobj)
    if _stale(dobj, [drv] + headers):
        cmds.append([CLANG, "-O1", "-g", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"] + SAN +
                    ["-c", drv, "-o", dobj])

    def run(cmd):
        if verbose:
            print("+", " ".join(cmd), flush=True)
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if r.returncode:
            raise RuntimeError(f"{' '.join(cmd)}\n{r.stdout[-4000:]}")

    jobs = max(1, min(len(cmds) or 1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(run, cmds))
    if cmds or not os.path.exists(EXE):
        run([CLANG] + SAN[:1] + ["-o", EXE + ".tmp"] + objs +
            ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
        os.replace(EXE + ".tmp", EXE)
    write_channels()
    return EXE


if __name__ == "__main__":
    print(build(verbose=True))
