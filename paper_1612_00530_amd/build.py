"""Build libspmvc.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libspmvc.so")
SOURCES = ["api.cpp", "tune.cpp", "scan.hip", "compress.hip", "spmv.hip", "cg.hip", "batched.hip", "symgs.hip", "reorder.hip"]
ARCH = os.environ.get("SPMVC_ARCH", "gfx950")

FLAGS = [
    "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # code object v5 loads on the HIP runtime torch brings as well as on the system one
    "-mcode-object-version=5",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


CHECK_BUILD = os.path.join(HERE, "_build_check")
CHECK_LIB = os.path.join(HERE, "libspmvc_check.so")


def _compile(src: str, check: bool = False) -> str:
    obj = os.path.join(CHECK_BUILD if check else BUILD, os.path.splitext(src)[0] + ".o")
    flags = FLAGS
    if check:
        # -O1: the bounds checks add a branch to every gather of the unrolled
        # kernel templates, which makes -O3 code generation take many times
        # longer; the checked build exists to test index arithmetic, which
        # does not depend on the optimisation level
        flags = [f if f != "-O3" else "-O1" for f in FLAGS] + ["-DSPMVC_CHECK"]
    cmd = [_hipcc(), *flags, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int = 6, verbose: bool = False, check: bool = False) -> str:
    """Compile every source for gfx950 and link libspmvc.so next to this file
    (check=True: the bounds-checked debug build, -DSPMVC_CHECK, as
    libspmvc_check.so)."""
    os.makedirs(CHECK_BUILD if check else BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda src: _compile(src, check), SOURCES))
    lib = CHECK_LIB if check else LIB
    tmp = lib + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-mcode-object-version=5", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    build(verbose=True, jobs=int(sys.argv[1]) if len(sys.argv) > 1 else 6, check="check" in sys.argv[2:])
