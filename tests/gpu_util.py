"""Helpers shared by the GPU tests: moving CSR inputs to the device, tolerances."""
import numpy as np

GAMMA_F64 = 2.0 ** -53
U_F32 = 2.0 ** -24


def torch_mod():
    import torch

    if not torch.cuda.is_available():
        import pytest

        pytest.skip("no GPU")
    return torch


def lib():
    """The GPU binding; fails loudly when the HIP library is not built."""
    import paper_1612_00530_amd as P

    P.load()
    return P


def to_dev(A):
    torch = torch_mod()
    return (torch.from_numpy(A.row_ptr).cuda(), torch.from_numpy(A.col).cuda(),
            torch.from_numpy(A.val).cuda())


def compress(A, **kw):
    P = lib()
    rp, col, val = to_dev(A)
    return P.compress(rp, col, val, n_cols=A.n_cols, **kw)


def row_scale(A, x):
    """sum_j |a_ij| |x_j| per row (the cancellation-safe normaliser of the SpMV error)."""
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
    with np.errstate(invalid="ignore"):  # 0 * inf in the special-value cases
        return np.bincount(rows, weights=np.abs(A.val) * np.abs(x[A.col]), minlength=A.n_rows)


def max_rel_err(A, x, y_gpu, y_ref):
    """max_i |y_i - yref_i| / sum_j |a_ij||x_j| over rows with a non-zero scale."""
    s = row_scale(A, x)
    d = np.abs(y_gpu - y_ref)
    nz = s > 0
    if np.any(d[~nz] != 0):
        return np.inf
    return float((d[nz] / s[nz]).max()) if nz.any() else 0.0


def same_bits(a, b):
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    return a.shape == b.shape and np.array_equal(a.view(np.uint8), b.view(np.uint8))
