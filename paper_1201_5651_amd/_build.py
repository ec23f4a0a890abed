"""Build step of the HIP library: compiles csrc/ for gfx950 into libpi.so
(in the package directory, so it travels with the tree).  Each translation
unit is compiled in its own hipcc process (in parallel), then linked."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpi.so")
SOURCES = ["kernels.hip", "engine.hip", "runtime.hip", "server.hip", "noalloc.hip"]
HEADERS = ["physics.h", "kernels.h", "engine.h", "arena.h"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are disabled for every HIP translation unit
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # every device atomic here is issued by one lane already; without the
    # wave-combining rewrite a returning atomic is waited for only where its
    # value is used (the persistent kernels claim their next tile early)
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-Wno-unused-command-line-argument",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(HERE, "..", "include")]
    with tempfile.TemporaryDirectory(prefix="pi_build_") as tmpd:
        procs, objs = [], []
        for src in sources():
            obj = os.path.join(tmpd, os.path.basename(src) + ".o")
            cmd = [hipcc] + HIPCC_FLAGS + inc + ["-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), file=sys.stderr)
            procs.append((src, subprocess.Popen(cmd)))
            objs.append(obj)
        failed = [s for s, p in procs if p.wait() != 0]
        if failed:
            raise RuntimeError("hipcc failed on " + ", ".join(failed))
        tmp = LIB + ".tmp"
        cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
