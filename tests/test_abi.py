"""The C-ABI library: it loads and exports every entry point include/spmvc.h declares.

Runs without a GPU (no compute calls).
"""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spmvc.h")
LIB = os.path.join(ROOT, "paper_1612_00530_amd", "libspmvc.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:spmvc_status|void|const char\s*\*|char\s*\*)\s*\*?\s*(\w+)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["spmv_compress", "spmv", "spmv_block", "cg_solve"]:
        assert required in names
    assert len(names) >= 12


CHECK_LIB = os.path.join(ROOT, "paper_1612_00530_amd", "libspmvc_check.so")


@pytest.mark.parametrize("path", [LIB, CHECK_LIB], ids=["release", "bounds_checked"])
def test_library_exports_every_declared_symbol(path):
    """The release library and the bounds-checked debug build (-DSPMVC_CHECK)
    export the same boundary."""
    if not os.path.exists(path):
        pytest.skip(os.path.basename(path) + " not built")
    lib = ctypes.CDLL(path)
    for name in declared_functions():
        assert hasattr(lib, name), name
    lib.spmvc_check_violations.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.spmvc_check_violations(None, None) == -1  # rejected on the host
    if path == LIB:  # the probe exists in checked builds only
        lib.spmvc_check_probe.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
        assert lib.spmvc_check_probe(3, 3, None) == -8
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (\w+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported


@pytest.mark.skipif(not os.path.exists(LIB), reason="libspmvc.so not built")
def test_status_strings_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.spmvc_status_string.restype = ctypes.c_char_p
    lib.spmvc_status_string.argtypes = [ctypes.c_int32]
    assert lib.spmvc_status_string(0) == b"ok"
    assert b"SPD" in lib.spmvc_status_string(-6)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libspmvc.so not built")
def test_null_arguments_rejected_on_host():
    """Host-side validation: no device work is issued for these calls."""
    lib = ctypes.CDLL(LIB)
    P = ctypes.c_void_p
    lib.spmv.argtypes = [P, ctypes.c_int32, P, P, P]
    lib.spmv_compress.argtypes = [ctypes.c_int64] * 3 + [P] * 6
    assert lib.spmv(None, 0, None, None, None) == -1
    assert lib.spmv_compress(4, 4, 0, None, None, None, None, None, None) == -1
    out = P()
    assert lib.spmv_compress(-1, 4, 0, None, None, None, None, None, ctypes.byref(out)) == -1
    lib.spmvc_last_error.restype = ctypes.c_char_p
    assert b"negative" in lib.spmvc_last_error()
    lib.spmv_set_block_mode.argtypes = [P, ctypes.c_int32]
    assert lib.spmv_set_block_mode(None, 1) == -1
    lib.spmv_set_config.argtypes = [P, ctypes.c_int32, ctypes.c_int32]
    assert lib.spmv_set_config(None, 512, 1) == -1
    lib.spmv_symgs.argtypes = [P, P, P, ctypes.c_int32, P]
    assert lib.spmv_symgs(None, None, None, 1, None) == -1
    # allocator hooks: both or neither
    alloc_t = ctypes.CFUNCTYPE(P, ctypes.c_size_t, P, P)
    free_t = ctypes.CFUNCTYPE(None, P, P, P)
    lib.spmvc_set_allocator.argtypes = [alloc_t, free_t, P]
    assert lib.spmvc_set_allocator(alloc_t(lambda n, s, c: None), free_t(), None) == -1
    assert lib.spmvc_set_allocator(alloc_t(), free_t(), None) == 0
    lib.spmvc_batched_config.argtypes = [P, P, P]
    assert lib.spmvc_batched_config(None, None, None) == -1
    lib.cg_solve_mg.argtypes = [P, P, ctypes.c_int32, P, P, P, P, P]
    stat = (ctypes.c_byte * 32)()
    levels = (P * 2)(None, None)
    assert lib.cg_solve_mg(None, None, 1, None, None, None, stat, None) == -1
    assert lib.cg_solve_mg(levels, None, 0, None, None, None, stat, None) == -1
    assert lib.cg_solve_mg(levels, None, 17, None, None, None, stat, None) == -1
    assert lib.cg_solve_mg(levels, None, 2, None, None, None, stat, None) == -1
    assert b"f2c" in lib.spmvc_last_error()
    assert lib.cg_solve_mg(levels, None, 1, None, None, None, stat, None) == -1
    assert b"handle" in lib.spmvc_last_error()
    lib.spmv_rcm.argtypes = [ctypes.c_int64, P, P, P, P]
    assert lib.spmv_rcm(-1, None, None, None, None) == -1
    assert lib.spmv_rcm(4, None, None, None, None) == -1
    assert lib.spmv_rcm(1 << 31, None, None, None, None) == -1
    lib.spmv_permute.argtypes = [ctypes.c_int64] + [P] * 8
    assert lib.spmv_permute(4, None, None, None, None, None, None, None, None) == -1


def test_binding_fails_loudly_without_library(tmp_path):
    import paper_1612_00530_amd as P

    with pytest.raises(ImportError):
        P.load(str(tmp_path / "missing.so"))
