"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* the oracle (oracle/oracle.c) built with both sanitizers and driven through
  SpMV, block SpMV, CG and the residual (tests/native/oracle_sanitize_driver.c);
* the library's C ABI layer (csrc/api.cpp) and autotuner (csrc/tune.cpp)
  built with both sanitizers on the host side only (device code unchanged)
  and linked with the library's other objects; every entry point is called
  with arguments its host-side checks reject (tests/native/abi_sanitize_driver.cpp).

Sanitizer errors abort the driver (no recovery), so a non-zero exit fails the test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
PKG = os.path.join(ROOT, "paper_1612_00530_amd")
BUILD = os.path.join(PKG, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
HOST_SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_drv")
    _run(["gcc", "-O1", "-g", *HOST_SAN, "-fopenmp", "-ffp-contract=off", "-o", exe,
          os.path.join(NATIVE, "oracle_sanitize_driver.c"), os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    r = _run([exe], env=SAN_ENV)
    assert "ok" in r.stdout


OTHER_OBJS = ["scan", "compress", "spmv", "cg", "batched", "symgs", "reorder"]


@pytest.mark.skipif(not all(os.path.exists(os.path.join(BUILD, o + ".o")) for o in OTHER_OBJS)
                    or not os.path.exists(os.path.join(ROCM, "bin", "hipcc")),
                    reason="library objects not built (run the package build first) or no ROCm compiler")
def test_abi_host_code_under_sanitizers(tmp_path):
    compiler = os.path.join(ROCM, "bin", "hipcc")
    # sanitizers for the host pass only: each flag behind -Xarch_host
    host_only = [f for flag in HOST_SAN for f in ("-Xarch_host", flag)]
    flags = ["-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-mcode-object-version=5",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *host_only]
    objs = []
    for src in (os.path.join(PKG, "csrc", "api.cpp"), os.path.join(PKG, "csrc", "tune.cpp"),
                os.path.join(NATIVE, "abi_sanitize_driver.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([compiler, *flags, "-c", src, "-o", obj])
        objs.append(obj)
    exe = str(tmp_path / "abi_drv")
    linker = os.path.join(ROCM, "llvm", "bin", "clang++")
    _run([linker, *HOST_SAN, "-o", exe, *objs, *[os.path.join(BUILD, o + ".o") for o in OTHER_OBJS],
          "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    r = _run([exe], env=SAN_ENV)
    assert "ok" in r.stdout
