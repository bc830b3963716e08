"""Builds libmsim.so (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmsim.so")
SOURCES = ["msim_kernels.hip", "msim_adjoint.hip", "msim_farrow.hip", "msim_host.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # packed FP32 VALU ops are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer (device code is built
# as usual: the flags apply to the host pass only).
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, sanitize: bool = False, out: str = LIB) -> str:
    """Compiles every source and links `out` (sanitize: the host code with ASan
    and UBSan, for CPU-side tests that preload the clang runtime)."""
    objs = []
    tag = ".san" if sanitize else ""
    extra = SANITIZE_FLAGS if sanitize else []
    cmds = []
    for src in SOURCES:
        obj = os.path.join(os.path.dirname(out), src.rsplit(".", 1)[0] + tag + ".%d.o" % os.getpid())
        cmds.append([HIPCC, "-x", "hip", "-c", *FLAGS, *extra, os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    # the sources compile side by side (one hipcc each)
    procs = []
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
    bad = [c for p, c in zip(procs, cmds) if p.wait() != 0]
    if bad:
        raise subprocess.CalledProcessError(1, bad[0])
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *extra, *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    for o in objs:
        os.remove(o)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
