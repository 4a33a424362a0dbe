"""Python binding of libspmvc: compressed SpMV and CG on MI355X (gfx950).

Argument marshalling only: every step of compression, SpMV and CG runs in the
HIP kernels of ``libspmvc.so`` behind the C ABI declared in
``include/spmvc.h``.  Torch tensors supply device memory and the current HIP
stream.  The library must be built (``paper_1612_00530_amd.build.build()``);
there is no CPU fallback, and importing this module without the library
raises at first use.
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "load", "compress", "Matrix", "cg_solve", "cg_solve_mg", "rcm", "permute", "SpmvcError",
    "FMT_ELL", "FMT_DT", "FMT_DIT", "FMT_DITV", "F64", "F32",
]

HERE = os.path.dirname(os.path.abspath(__file__))
# SPMVC_LIBRARY names another build of the library to load instead (the
# bounds-checked libspmvc_check.so, for instance)
LIB_PATH = os.environ.get("SPMVC_LIBRARY") or os.path.join(HERE, "libspmvc.so")
CHECK_LIB_PATH = os.path.join(HERE, "libspmvc_check.so")

FMT_ELL, FMT_DT, FMT_DIT, FMT_DITV, FMT_AUTO, FMT_BMASK = 0, 1, 2, 3, 4, 5
F64, F32 = 0, 1
_FMT_NAMES = {"ELL": FMT_ELL, "DT": FMT_DT, "DIT": FMT_DIT, "DITV": FMT_DITV, "AUTO": FMT_AUTO,
              "BMASK": FMT_BMASK}

ARR = {
    "ELL_VAL": 0, "ELL_COL": 1, "DT_S": 2, "IDS": 3, "T": 4, "PAT_OFF": 5, "PAT_LEN": 6,
    "RAW": 7, "RAW_SLICE": 8, "ESC_ROWS": 9, "ESC_PTR": 10, "ESC_COL": 11, "ESC_VAL": 12, "V": 13,
    "PAT_T": 14, "BM_D": 15, "BM_MASK": 16, "BM_VMASK": 17,
}

EXPORTED = [
    "spmv_compress", "spmv", "spmv_block", "cg_solve", "cg_solve_noalloc", "cg_solve_mg", "spmv_decompress", "spmv_info",
    "spmv_get_array", "spmv_set_config", "spmv_set_block_mode", "spmv_tune", "spmv_symgs", "spmv_colors",
    "spmv_color_order", "spmvc_check_violations", "spmvc_check_probe",
    "spmvc_batched_config", "spmvc_set_allocator", "spmv_rcm", "spmv_permute", "spmv_free", "spmvc_status_string",
    "spmvc_last_error",
]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
_alloc_hooks = []  # every installed pair of ctypes callbacks, kept alive: buffers return to their own


class SpmvcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"spmvc status {status}: {msg}")
        self.status = status


class CompressOpts(ctypes.Structure):
    _fields_ = [("fmt", ctypes.c_int32), ("k_max", ctypes.c_int32), ("p_max", ctypes.c_int32),
                ("min_pattern_rows", ctypes.c_int32), ("f32_shadow", ctypes.c_int32)]


class CgOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("inner_rtol", ctypes.c_double), ("max_outer", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("batched", ctypes.c_int32)]


class CgStat(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("outer_iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("relres_true", ctypes.c_double),
                ("relres_recursive", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("fmt", ctypes.c_int32), ("K", ctypes.c_int32), ("P", ctypes.c_int32),
                ("id_bytes", ctypes.c_int32), ("width", ctypes.c_int32), ("max_raw", ctypes.c_int32),
                ("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("n_escape_rows", ctypes.c_int64), ("n_escape_nnz", ctypes.c_int64),
                ("n_raw", ctypes.c_int64), ("bytes_stream", ctypes.c_int64),
                ("bytes_ell", ctypes.c_int64), ("bytes_paper", ctypes.c_int64),
                ("lds_windows", ctypes.c_int32), ("rows_per_block", ctypes.c_int32),
                ("V", ctypes.c_double * 15), ("kernel", ctypes.c_int32), ("kernel_f32", ctypes.c_int32),
                ("rows_per_block_f32", ctypes.c_int32), ("block_split", ctypes.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libspmvc.so (raises ImportError if it has not been built)."""
    global _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1612_00530_amd.build.build()")
    if _lib is not None and path == LIB_PATH:
        return _lib
    # torch first: its HIP runtime (soname libamdhip64.so.7) then also serves this
    # library, so the process holds one HIP runtime, not two.
    import torch  # noqa: F401

    lib = ctypes.CDLL(path)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.spmv_compress.argtypes = [i64, i64, i64, P, P, P, ctypes.POINTER(CompressOpts), P, ctypes.POINTER(P)]
    lib.spmv.argtypes = [P, i32, P, P, P]
    lib.spmv_block.argtypes = [P, i32, i32, P, i64, P, i64, P]
    lib.cg_solve.argtypes = [ctypes.POINTER(P), i32, i32, ctypes.POINTER(P), ctypes.POINTER(P),
                             ctypes.POINTER(CgOpts), ctypes.POINTER(CgStat), P]
    lib.cg_solve_noalloc.argtypes = [P, P, P, ctypes.POINTER(CgOpts), ctypes.POINTER(CgStat), P]
    lib.cg_solve_mg.argtypes = [ctypes.POINTER(P), ctypes.POINTER(P), i32, P, P, ctypes.POINTER(CgOpts),
                                ctypes.POINTER(CgStat), P]
    lib.spmv_decompress.argtypes = [P, P, P, P, P]
    lib.spmv_rcm.argtypes = [i64, P, P, P, P]
    lib.spmv_permute.argtypes = [i64, P, P, P, P, P, P, P, P]
    lib.spmv_info.argtypes = [P, ctypes.POINTER(Info)]
    lib.spmv_get_array.argtypes = [P, i32, P, ctypes.POINTER(i64), P]
    lib.spmv_set_config.argtypes = [P, i32, i32]
    lib.spmv_set_block_mode.argtypes = [P, i32]
    lib.spmv_tune.argtypes = [P, i32, i32, P, ctypes.POINTER(i32), ctypes.POINTER(i32),
                              ctypes.POINTER(ctypes.c_double)]
    lib.spmv_symgs.argtypes = [P, P, P, i32, P]
    lib.spmv_colors.argtypes = [P, ctypes.POINTER(i32), P, P]
    lib.spmv_color_order.argtypes = [P, ctypes.POINTER(P), P, P]
    lib.spmvc_check_violations.argtypes = [ctypes.POINTER(i64), ctypes.POINTER(i32)]
    lib.spmvc_check_probe.argtypes = [i64, i64, P]
    lib.spmvc_batched_config.argtypes = [ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
    lib.spmvc_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, P]
    lib.spmv_free.argtypes = [P]
    lib.spmv_free.restype = None
    lib.spmvc_status_string.argtypes = [i32]
    lib.spmvc_status_string.restype = ctypes.c_char_p
    lib.spmvc_last_error.restype = ctypes.c_char_p
    for name in ["spmv_compress", "spmv", "spmv_block", "cg_solve", "cg_solve_mg", "spmv_decompress", "spmv_info",
                 "spmv_get_array", "spmv_set_config", "spmv_set_block_mode", "spmv_tune", "spmv_symgs",
                 "spmv_colors", "spmvc_batched_config", "spmvc_set_allocator", "spmv_rcm", "spmv_permute"]:
        getattr(lib, name).restype = ctypes.c_int
    if path == LIB_PATH:
        _lib = lib
    return lib


def _check(st: int):
    if st != 0:
        msg = load().spmvc_last_error().decode() or load().spmvc_status_string(st).decode()
        raise SpmvcError(st, msg)


def _stream(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype, name):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr() if t.numel() else 0)


def _dev_rows(t, dtype, name):
    """Device pointer of a row-major 2-D block whose rows may be padded (leading
    dimension stride(0) >= number of columns, unit column stride)."""
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() != 2 or (t.shape[1] > 1 and t.stride(1) != 1) or t.stride(0) < t.shape[1]:
        raise ValueError(f"{name} must be a row-major block (unit column stride, leading dimension >= columns)")
    return ctypes.c_void_p(t.data_ptr() if t.numel() else 0)


class Matrix:
    """A compressed matrix owned by libspmvc (released by ``free`` or garbage collection)."""

    def __init__(self, handle, n_rows, n_cols, nnz):
        self._h = handle
        self.n_rows, self.n_cols, self.nnz = n_rows, n_cols, nnz

    @property
    def handle(self):
        return self._h

    def free(self):
        if self._h:
            load().spmv_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def info(self) -> dict:
        inf = Info()
        _check(load().spmv_info(self._h, ctypes.byref(inf)))
        d = {f: getattr(inf, f) for f, _ in Info._fields_ if f != "V"}
        d["V"] = [inf.V[i] for i in range(inf.K)]
        d["fmt_name"] = {0: "ELL", 1: "DT", 2: "DIT", 3: "DITV", 5: "BMASK"}[inf.fmt]
        names = {0: "k_spmv_direct", 1: "k_dit_lds", 2: "k_dit_reg", 3: "k_dit_march", 4: "k_bmask_lds"}
        d["kernel_name"] = names[inf.kernel]
        d["kernel_name_f32"] = names[inf.kernel_f32]
        return d

    def spmv(self, x, y=None, dtype=None, stream=None):
        """y = A x on the GPU (x, y: float64 or float32 CUDA tensors)."""
        import torch

        dtype = dtype or x.dtype
        dt = F64 if dtype == torch.float64 else F32
        if x.shape != (self.n_cols,):
            raise ValueError("x has the wrong shape")
        if y is None:
            y = torch.empty(self.n_rows, dtype=dtype, device=x.device)
        elif y.shape != (self.n_rows,):
            raise ValueError("y has the wrong shape")
        _check(load().spmv(self._h, dt, _dev(x, dtype, "x"), _dev(y, dtype, "y"), _stream(stream)))
        return y

    def spmv_block(self, X, Y=None, stream=None):
        """Y = A X for row-interleaved X of shape (n_cols, nrhs)."""
        import torch

        dt = F64 if X.dtype == torch.float64 else F32
        if X.dim() != 2 or X.shape[0] != self.n_cols:
            raise ValueError("X must be (n_cols, nrhs)")
        nrhs = X.shape[1]
        if Y is None:
            Y = torch.empty((self.n_rows, nrhs), dtype=X.dtype, device=X.device)
        if Y.shape != (self.n_rows, nrhs):
            raise ValueError("Y must be (n_rows, nrhs)")
        _check(load().spmv_block(self._h, dt, nrhs, _dev_rows(X, X.dtype, "X"), max(X.stride(0), nrhs),
                                 _dev_rows(Y, X.dtype, "Y"), max(Y.stride(0), nrhs), _stream(stream)))
        return Y

    def symgs(self, b, x=None, sweeps=1, stream=None):
        """`sweeps` multicolor symmetric Gauss-Seidel sweeps on A x = b (FP64); x is
        updated in place (a zero vector when None) and returned."""
        import torch

        if x is None:
            x = torch.zeros(self.n_rows, dtype=torch.float64, device=b.device)
        if b.numel() != self.n_rows or x.numel() != self.n_rows:
            raise ValueError("b and x must have n_rows elements")
        _check(load().spmv_symgs(self._h, _dev(b, torch.float64, "b"), _dev(x, torch.float64, "x"), int(sweeps),
                                 _stream(stream)))
        return x

    def colors(self):
        """(number of colors, int32 CUDA tensor of each row's color) of the SymGS coloring."""
        import torch

        nc = ctypes.c_int32()
        col = torch.empty(max(self.n_rows, 1), dtype=torch.int32, device="cuda")
        _check(load().spmv_colors(self._h, ctypes.byref(nc), ctypes.c_void_p(col.data_ptr()), _stream()))
        return nc.value, col[: self.n_rows]

    def color_order(self):
        """(B, perm): B = P A P^T with the rows of each SymGS color contiguous (a new
        Matrix; its coloring is the one induced from this matrix's), perm an int32
        CUDA tensor with perm[k] = the row of this matrix that is row k of B."""
        import torch

        perm = torch.empty(max(self.n_rows, 1), dtype=torch.int32, device="cuda")
        h = ctypes.c_void_p()
        _check(load().spmv_color_order(self._h, ctypes.byref(h), ctypes.c_void_p(perm.data_ptr()), _stream()))
        return Matrix(h, self.n_rows, self.n_cols, self.nnz), perm[: self.n_rows]

    def decompress(self):
        import torch

        dev = torch.device("cuda")
        rp = torch.empty(self.n_rows + 1, dtype=torch.int64, device=dev)
        col = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=dev)
        val = torch.empty(max(self.nnz, 1), dtype=torch.float64, device=dev)
        _check(load().spmv_decompress(self._h, _dev(rp, torch.int64, "rp"), ctypes.c_void_p(col.data_ptr()),
                                      ctypes.c_void_p(val.data_ptr()), _stream()))
        return rp, col[: self.nnz], val[: self.nnz]

    def array(self, name: str):
        """Copy of an internal array as a uint8 CUDA tensor (layout: see include/spmvc.h)."""
        import torch

        nb = ctypes.c_int64()
        _check(load().spmv_get_array(self._h, ARR[name], None, ctypes.byref(nb), _stream()))
        out = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        if nb.value:
            _check(load().spmv_get_array(self._h, ARR[name], ctypes.c_void_p(out.data_ptr()),
                                         ctypes.byref(nb), _stream()))
        return out

    def set_config(self, rows_per_block=0, lds=-1):
        _check(load().spmv_set_config(self._h, rows_per_block, lds))

    def set_block_mode(self, mode):
        _check(load().spmv_set_block_mode(self._h, mode))

    def tune(self, dtype=None, nrhs=1):
        import torch

        dt = F32 if dtype == torch.float32 else F64
        rows, lds, us = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(load().spmv_tune(self._h, dt, nrhs, _stream(), ctypes.byref(rows), ctypes.byref(lds),
                                ctypes.byref(us)))
        return {"rows_per_block": rows.value, "lds": lds.value, "us": us.value}


def compress(row_ptr, col, val, n_cols=None, fmt="DIT", k_max=15, p_max=65535, min_pattern_rows=2,
             f32_shadow=True, stream=None) -> Matrix:
    """Compress a CSR matrix held in CUDA tensors (int64 row_ptr, int32 col, float64 val)."""
    import torch

    n_rows = row_ptr.numel() - 1
    nnz = col.numel()
    if n_cols is None:
        raise ValueError("n_cols is required")
    o = CompressOpts(_FMT_NAMES[fmt] if isinstance(fmt, str) else int(fmt), k_max, p_max, min_pattern_rows,
                     1 if f32_shadow else 0)
    h = ctypes.c_void_p()
    _check(load().spmv_compress(n_rows, int(n_cols), nnz, _dev(row_ptr, torch.int64, "row_ptr"),
                                _dev(col, torch.int32, "col"), _dev(val, torch.float64, "val"),
                                ctypes.byref(o), _stream(stream), ctypes.byref(h)))
    return Matrix(h, n_rows, int(n_cols), nnz)


def cg_solve(mats, bs, xs=None, rtol=1e-10, max_iter=10000, mode=0, inner_rtol=1e-5, max_outer=20,
             check_every=16, nrhs=1, batched=2, stream=None):
    """CG on one or more systems; bs/xs: lists of CUDA float64 tensors (n,) or (n, nrhs)."""
    import torch

    if isinstance(mats, Matrix):
        mats, bs = [mats], [bs]
        xs = [xs] if xs is not None else None
    n_sys = len(mats)
    if xs is None:
        xs = [torch.empty_like(b) for b in bs]
    H = (ctypes.c_void_p * n_sys)(*[m.handle for m in mats])
    B = (ctypes.c_void_p * n_sys)(*[_dev(b, torch.float64, "b").value for b in bs])
    X = (ctypes.c_void_p * n_sys)(*[_dev(x, torch.float64, "x").value for x in xs])
    o = CgOpts(rtol, max_iter, mode, inner_rtol, max_outer, check_every, batched)
    stats = (CgStat * (n_sys * nrhs))()
    st = load().cg_solve(H, n_sys, nrhs, B, X, ctypes.byref(o), stats, _stream(stream))
    out = [{"iters": s.iters, "outer_iters": s.outer_iters, "status": s.status,
            "relres_true": s.relres_true, "relres_recursive": s.relres_recursive} for s in stats]
    return st, xs, out


def cg_solve_noalloc(mat, b, x=None, rtol=1e-10, max_iter=10000, check_every=16, stream=None):
    """FP64 CG of one system through the library's allocation-free entry point
    (every buffer of the solve in its static device region).  b, x: CUDA
    float64 vectors; x is allocated here when not given."""
    import torch

    if x is None:
        x = torch.empty_like(b)
    o = CgOpts(rtol, max_iter, 0, 1e-5, 20, check_every, 0)
    stat = (CgStat * 1)()
    st = load().cg_solve_noalloc(mat.handle, _dev(b, torch.float64, "b"), _dev(x, torch.float64, "x"),
                                 ctypes.byref(o), stat, _stream(stream))
    s = stat[0]
    return st, x, {"iters": s.iters, "status": s.status, "relres_true": s.relres_true,
                   "relres_recursive": s.relres_recursive}


def cg_solve_mg(levels, f2c, b, x=None, rtol=1e-10, max_iter=10000, check_every=16, stream=None):
    """CG on levels[0] x = b preconditioned by one multigrid V-cycle per iteration.
    levels: list of Matrix (finest first); f2c: list of len(levels) - 1 CUDA int32
    tensors (fine row of each coarse row); b, x: CUDA float64 vectors."""
    import torch

    n_lev = len(levels)
    if len(f2c) != n_lev - 1:
        raise ValueError("f2c needs one map per coarse level")
    if x is None:
        x = torch.empty_like(b)
    H = (ctypes.c_void_p * n_lev)(*[m.handle for m in levels])
    F = (ctypes.c_void_p * max(n_lev - 1, 1))(*[_dev(f, torch.int32, "f2c").value for f in f2c])
    o = CgOpts(rtol, max_iter, 0, 1e-5, 20, check_every, 0)
    stat = (CgStat * 1)()
    st = load().cg_solve_mg(H, F, n_lev, _dev(b, torch.float64, "b"), _dev(x, torch.float64, "x"),
                            ctypes.byref(o), stat, _stream(stream))
    s = stat[0]
    return st, x, {"iters": s.iters, "status": s.status, "relres_true": s.relres_true,
                   "relres_recursive": s.relres_recursive}


def rcm(row_ptr, col, stream=None):
    """Reverse Cuthill-McKee permutation (CUDA int32 tensor, perm[new] = old) of a
    structurally symmetric CSR matrix given as CUDA int64 row_ptr / int32 col."""
    import torch

    n = row_ptr.numel() - 1
    perm = torch.empty(max(n, 0), dtype=torch.int32, device=row_ptr.device)
    _check(load().spmv_rcm(n, _dev(row_ptr, torch.int64, "row_ptr"), _dev(col, torch.int32, "col"),
                           _dev(perm, torch.int32, "perm"), _stream(stream)))
    return perm


def permute(row_ptr, col, val, perm, stream=None):
    """B = P A P^T of a CSR matrix (CUDA tensors); returns (row_ptr, col, val) of B."""
    import torch

    n = row_ptr.numel() - 1
    out_rp = torch.empty_like(row_ptr)
    out_col = torch.empty_like(col)
    out_val = torch.empty_like(val)
    _check(load().spmv_permute(n, _dev(row_ptr, torch.int64, "row_ptr"), _dev(col, torch.int32, "col"),
                               _dev(val, torch.float64, "val"), _dev(perm, torch.int32, "perm"),
                               _dev(out_rp, torch.int64, "out_row_ptr"), _dev(out_col, torch.int32, "out_col"),
                               _dev(out_val, torch.float64, "out_val"), _stream(stream)))
    return out_rp, out_col, out_val


def batched_config():
    """The SpMV configuration the last batched cg_solve chose: {"form", "chunk", "us"}
    (form 0 window-phased, 1 lane groups with rhs pairs, 2 lane groups; -1 before any;
    -2 when that solve took the one-after-another path instead)."""
    f, c, us = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _check(load().spmvc_batched_config(ctypes.byref(f), ctypes.byref(c), ctypes.byref(us)))
    return {"form": f.value, "chunk": c.value, "us": us.value}


def check_violations():
    """(violations recorded since the last call, whether this library is the
    bounds-checked build)."""
    n, checked = ctypes.c_int64(), ctypes.c_int32()
    _check(load().spmvc_check_violations(ctypes.byref(n), ctypes.byref(checked)))
    return n.value, bool(checked.value)


def check_probe(i, n):
    """Checked builds: pass index i against [0, n) through the kernels' bounds
    check on the device (a violation is then reported by check_violations)."""
    _check(load().spmvc_check_probe(int(i), int(n), _stream()))


def use_torch_allocator(enable=True):
    """Route the library's device allocations through torch's caching allocator
    (spmvc_set_allocator), or back to hipMalloc / hipFree with enable=False.
    Buffers already allocated go back to the allocator that made them."""
    import torch

    if not enable:
        _check(load().spmvc_set_allocator(_ALLOC_FN(), _FREE_FN(), None))
        return

    def _alloc(nbytes, stream, ctx):
        return torch.cuda.caching_allocator_alloc(int(nbytes))

    def _free(ptr, stream, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    hooks = (_ALLOC_FN(_alloc), _FREE_FN(_free))
    _alloc_hooks.append(hooks)
    _check(load().spmvc_set_allocator(hooks[0], hooks[1], None))
