"""CPU oracle for the compressed-SpMV / CG path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU
library (``paper_1612_00530_amd``) and never imports it.

* ``spmv``, ``spmv_block``, ``cg``, ``relres`` -- thin ctypes wrappers over
  ``oracle.c`` (plain FP64 CSR SpMV and textbook CG, see that file).
* ``codec`` -- the reference codec for the paper's compression schemes
  (Section V: value table V, sorted column list S_i, terminal indices T_i,
  displacement-pattern table), written with numpy.
* ``gs`` -- multicolor symmetric Gauss-Seidel (the SymGS kernel of Table I),
  its greedy row-order coloring, and CG preconditioned by one sweep or by a
  multigrid V-cycle, written with numpy.
* ``reorder`` -- reverse Cuthill-McKee reordering and the symmetric
  permutation B = P A P^T (the reordering Section V proposes after Table II).

Pin status: ``spmv``/``spmv_block`` are pinned by dense brute force and by the
stencil's closed forms; ``cg`` by ``numpy.linalg.solve`` on small systems, by
x* = 1 for b = A*1 and by Krylov iteration-count bounds; ``relres`` two-sidedly
by closed forms (x = 0 gives 1; x = 1 + delta e_k against b = A*1 gives
delta ||A e_k|| / ||A*1||, counted from the grid) and by the dense definition; ``codec`` by the
paper's Fig. 1 example, its byte counts, lossless round trip and a
decoded-walk SpMV; ``gs`` by the stencil's parity coloring and by the
matrix-splitting form of Gauss-Seidel solved with dense triangular solves,
its V-cycle by the dense operator form; ``reorder`` by closed forms (paths,
stars), a hand-numbered example and a level-by-level formulation.
Nothing here is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (FP contraction off) into liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.oracle_spmv.argtypes = [i64, P, P, P, P, P]
        lib.oracle_spmv.restype = None
        lib.oracle_spmv_block.argtypes = [i64, P, P, P, ctypes.c_int32, P, i64, P, i64]
        lib.oracle_spmv_block.restype = None
        lib.oracle_cg.argtypes = [i64, P, P, P, P, P, ctypes.c_double, ctypes.c_int32, P, P]
        lib.oracle_cg.restype = ctypes.c_int
        lib.oracle_relres.argtypes = [i64, P, P, P, P, P]
        lib.oracle_relres.restype = ctypes.c_double
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr_arrays(A):
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(A.col, dtype=np.int32)
    val = np.ascontiguousarray(A.val, dtype=np.float64)
    return rp, col, val


def threads() -> int:
    """Number of OpenMP threads the oracle's SpMV uses."""
    return int(_load().oracle_threads())


def set_threads(t: int) -> None:
    _load().oracle_set_threads(int(t))


def spmv(A, x) -> np.ndarray:
    """y = A x (Eq. 1), FP64, each row summed in ascending column order."""
    rp, col, val = _csr_arrays(A)
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.shape[0] != A.n_cols:
        raise ValueError("x has wrong length")
    y = np.empty(A.n_rows, dtype=np.float64)
    _load().oracle_spmv(A.n_rows, _p(rp), _p(col), _p(val), _p(x), _p(y))
    return y


def spmv_block(A, X) -> np.ndarray:
    """Y = A X for X of shape (n_cols, nrhs), row-interleaved (C order)."""
    rp, col, val = _csr_arrays(A)
    X = np.ascontiguousarray(X, dtype=np.float64)
    if X.ndim != 2 or X.shape[0] != A.n_cols:
        raise ValueError("X must be (n_cols, nrhs)")
    nrhs = X.shape[1]
    Y = np.empty((A.n_rows, nrhs), dtype=np.float64)
    _load().oracle_spmv_block(A.n_rows, _p(rp), _p(col), _p(val), nrhs, _p(X), nrhs, _p(Y), nrhs)
    return Y


def cg(A, b, rtol: float = 1e-10, max_iter: int = 100000):
    """Unpreconditioned CG from x0 = 0.  Returns (x, status, iters, relres_recursive)."""
    if A.n_rows != A.n_cols:
        raise ValueError("CG needs a square matrix")
    rp, col, val = _csr_arrays(A)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.empty(A.n_rows, dtype=np.float64)
    it = np.zeros(1, dtype=np.int32)
    rel = np.zeros(1, dtype=np.float64)
    st = _load().oracle_cg(A.n_rows, _p(rp), _p(col), _p(val), _p(b), _p(x),
                           float(rtol), int(max_iter), _p(it), _p(rel))
    return x, int(st), int(it[0]), float(rel[0])


def relres(A, b, x) -> float:
    """True FP64 relative residual ||b - A x|| / ||b||."""
    rp, col, val = _csr_arrays(A)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    return float(_load().oracle_relres(A.n_rows, _p(rp), _p(col), _p(val), _p(b), _p(x)))
