"""Build the HIP library libshell_hip.so (gfx950) in-tree with hipcc.

Every source under csrc/ is compiled as HIP for gfx950 and linked into one shared library that
exports the C ABI of include/shell.h.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libshell_hip.so")
SOURCES = ["host_mesh.cpp", "precompute.hip", "forces.hip", "membrane.hip", "hessian.hip", "solver.hip", "capi.cpp"]
ARCH = os.environ.get("SHELL_OFFLOAD_ARCH", "gfx950")

CFLAGS = [
    "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-fPIC",
    "-munsafe-fp-atomics",
    # packed FP32 instructions stay off: plain scalar FP32 code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-function",
]


# the membrane step's host side is a C++20 coroutine (resumed as its device values land)
STD = {"membrane.hip": "-std=c++20"}


def hipcc() -> str:
    return os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")


def build(verbose: bool = False, defines=(), lib: str = LIB, obj: str = OBJ) -> str:
    """Compile and link; `defines` are extra -D tunables (kernel batch sizes), `lib` the output path."""
    os.makedirs(obj, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        o = os.path.join(obj, os.path.splitext(src)[0] + ".o")
        objs.append(o)
        cmd = [hipcc(), *CFLAGS, STD.get(src, "-std=c++17"), *[f"-D{d}" for d in defines], "-c",
               os.path.join(CSRC, src), "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass does not know the packed-fp32 feature; that warning is harmless
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if p.returncode != 0:
            failed.append(src)
            print(text, file=sys.stderr)
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        raise RuntimeError(f"hipcc failed for {failed}")
    tmp = lib + ".tmp"
    subprocess.run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
