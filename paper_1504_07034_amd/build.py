"""Build step of the LBRS library: hipcc for gfx950 -> liblbrs.so (in-tree)."""
from __future__ import annotations

import glob
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbrs.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed FP32 instructions stay off on these boxes
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def sources():
    """HIP sources, and the plain C++ host checks (lbrs_host.cpp)."""
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


OBJ = os.path.join(ROOT, "_build", "obj")


def build(verbose: bool = False, extra=None, jobs: int | None = None) -> str:
    """Compile every source of the library into liblbrs.so (always rebuilds):
    one hipcc per source file, in parallel, then one link."""
    os.makedirs(OBJ, exist_ok=True)
    compile_flags = [f for f in FLAGS if f != "-shared"]

    def one(src):
        obj = os.path.join(OBJ, os.path.basename(src) + ".o")
        cmd = [HIPCC, *compile_flags, *(extra or []), "-I", os.path.join(ROOT, "include"), "-c",
               src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        return obj

    srcs = sources()
    n = jobs or min(len(srcs), max(1, (os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=n) as ex:
        objs = list(ex.map(one, srcs))
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
