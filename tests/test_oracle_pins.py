"""Pins of the CPU oracle's SpMV and of the synthetic stencil matrices.

Every check here is against something other than the oracle itself: a dense
matrix built from the stencil's Kronecker closed form, the row-sum closed form
A*1 = 26 - (#neighbours), the stencil's analytic eigenpairs, symmetry and
diagonal dominance.
"""
import numpy as np
import pytest

import oracle
from synthetic import CSR, stencil27, stencil27_irregular, uniform_vector


def tridiag_ones(m):
    return np.eye(m) + np.eye(m, k=1) + np.eye(m, k=-1)


def dense_closed_form(nx, ny, nz):
    """A = 27 I - T_z (x) T_y (x) T_x, T_m = tridiag(1, 1, 1): the HPCG 27-point matrix."""
    K = np.kron(np.kron(tridiag_ones(nz), tridiag_ones(ny)), tridiag_ones(nx))
    return 27.0 * np.eye(nx * ny * nz) - K


def brute_force(D, x):
    """Dense y = D x, columns added one at a time in ascending order."""
    s = np.zeros(D.shape[0])
    for j in range(D.shape[1]):
        s = s + D[:, j] * x[j]
    return s


def to_dense(A):
    D = np.zeros((A.n_rows, A.n_cols))
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
    D[rows, A.col] = A.val
    return D


@pytest.mark.parametrize("grid", [(5, 4, 3), (16, 16, 16), (1, 3, 4), (2, 5, 7)])
def test_generator_matches_kronecker_closed_form(grid):
    A = stencil27(*grid)
    D = dense_closed_form(*grid)
    assert np.array_equal(to_dense(A), D)
    # columns strictly ascending within every row
    for i in range(0, A.n_rows, max(1, A.n_rows // 97)):
        c = A.col[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0)


def test_spmv_equals_dense_brute_force_16cubed():
    """The 16^3 workload itself: oracle y = A x bit-equals dense brute force (same order)."""
    A = stencil27(16, 16, 16)
    D = dense_closed_form(16, 16, 16)
    x = uniform_vector(A.n_cols, seed=0)
    y = oracle.spmv(A, x)
    assert np.array_equal(y, brute_force(D, x))


def test_spmv_block_equals_columnwise():
    A = stencil27(9, 7, 5)
    D = dense_closed_form(9, 7, 5)
    X = np.stack([uniform_vector(A.n_cols, seed=s) for s in range(8)], axis=1)
    Y = oracle.spmv_block(A, X)
    for r in range(8):
        assert np.array_equal(Y[:, r], brute_force(D, X[:, r]))


def test_spmv_nonsymmetric_catches_transpose():
    """A nonsymmetric random CSR: oracle equals D x and differs from D^T x."""
    rng = np.random.default_rng(5)
    n_rows, n_cols = 40, 55
    D = np.where(rng.random((n_rows, n_cols)) < 0.2, rng.uniform(-3, 3, (n_rows, n_cols)), 0.0)
    rp = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum((D != 0).sum(axis=1), out=rp[1:])
    r, c = np.nonzero(D)
    A = CSR(n_rows, n_cols, rp, c, D[r, c])
    x = rng.uniform(-1, 1, n_cols)
    y = oracle.spmv(A, x)
    assert np.array_equal(y, brute_force(D, x))
    Dsq = D[:, :n_rows]
    Asq_rows = np.nonzero(Dsq)
    rp2 = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum((Dsq != 0).sum(axis=1), out=rp2[1:])
    Asq = CSR(n_rows, n_rows, rp2, Asq_rows[1], Dsq[Asq_rows])
    xs = x[:n_rows]
    assert not np.allclose(oracle.spmv(Asq, xs), Dsq.T @ xs)


def neighbour_count(nx, ny, nz):
    i = np.arange(nx * ny * nz)
    ix, iy, iz = i % nx, (i // nx) % ny, i // (nx * ny)

    def span(c, m):
        return 1 + (c > 0) + (c < m - 1)

    return span(ix, nx) * span(iy, ny) * span(iz, nz) - 1


@pytest.mark.parametrize("grid", [(16, 16, 16), (104, 104, 104)])
def test_row_sum_closed_form(grid):
    """A*1 = 26 - (#neighbours); at 104^3 it takes the values {0, 9, 15, 19}."""
    A = stencil27(*grid)
    y = oracle.spmv(A, np.ones(A.n_cols))
    expect = 26.0 - neighbour_count(*grid)
    assert np.array_equal(y, expect)
    if grid[0] >= 3:
        assert set(np.unique(y).tolist()) == {0.0, 9.0, 15.0, 19.0}
    assert A.nnz == (3 * grid[0] - 2) * (3 * grid[1] - 2) * (3 * grid[2] - 2)


@pytest.mark.parametrize("grid,ks", [((16, 16, 16), (1, 2, 3)), ((12, 9, 7), (3, 1, 5)),
                                     ((104, 104, 104), (1, 1, 1))])
def test_eigenpair_closed_form(grid, ks):
    """A v = lambda v with v = (x) sin(k pi i / (n+1)), lambda = 27 - prod(1 + 2 cos(k pi/(n+1)))."""
    nx, ny, nz = grid
    A = stencil27(*grid)
    vs, lam_t = [], 1.0
    for m, k in zip(grid, ks):
        th = k * np.pi / (m + 1)
        vs.append(np.sin(th * np.arange(1, m + 1)))
        lam_t *= 1.0 + 2.0 * np.cos(th)
    v = np.kron(np.kron(vs[2], vs[1]), vs[0])
    lam = 27.0 - lam_t
    r = oracle.spmv(A, v) - lam * v
    assert np.abs(r).max() <= 1e-13 * 54.0 * np.abs(v).max()


def test_symmetry_and_dominance_stencil():
    A = stencil27(11, 6, 9)
    D = to_dense(A)
    assert np.array_equal(D, D.T)
    off = np.abs(D).sum(axis=1) - np.abs(np.diag(D))
    assert np.all(np.diag(D) >= off)  # weak: equality on interior rows
    assert np.any(np.diag(D) == off)


def test_irregular_symmetric_strictly_dominant_spd():
    A = stencil27_irregular(10, 9, 8, seed=3)
    D = to_dense(A)
    assert np.array_equal(D.view(np.uint64), D.T.view(np.uint64))
    d = np.diag(D)
    off = np.abs(D).sum(axis=1) - np.abs(d)
    assert np.all(d > off)
    assert np.linalg.eigvalsh(D).min() > 0
    full = stencil27(10, 9, 8)
    removed = 1.0 - (A.nnz - A.n_rows) / (full.nnz - full.n_rows)
    assert 0.02 < removed < 0.09
    offv = D[(D != 0) & ~np.eye(A.n_rows, dtype=bool)]
    assert offv.min() >= -1.5 and offv.max() <= -0.5
    # the removal is seeded: same seed -> same matrix, other seed -> other matrix
    B = stencil27_irregular(10, 9, 8, seed=3)
    C = stencil27_irregular(10, 9, 8, seed=4)
    assert np.array_equal(A.col, B.col) and np.array_equal(A.val, B.val)
    assert not (A.nnz == C.nnz and np.array_equal(A.col, C.col))


def test_spmv_irregular_brute_force():
    A = stencil27_irregular(9, 8, 7, seed=1)
    D = to_dense(A)
    x = uniform_vector(A.n_cols, seed=2)
    assert np.array_equal(oracle.spmv(A, x), brute_force(D, x))


def test_spmv_special_values_propagate():
    """Inf/NaN in x reach exactly the rows whose pattern touches them."""
    A = stencil27(6, 6, 6)
    x = np.ones(A.n_cols)
    x[100] = np.nan
    y = oracle.spmv(A, x)
    D = dense_closed_form(6, 6, 6)
    touched = D[:, 100] != 0
    assert np.all(np.isnan(y[touched]))
    assert not np.any(np.isnan(y[~touched]))


def test_empty_and_ragged_rows():
    rp = np.array([0, 0, 3, 3, 4, 4], dtype=np.int64)
    A = CSR(5, 7, rp, [0, 3, 6, 2], [1.0, -2.0, 0.5, 4.0])
    x = np.arange(7, dtype=np.float64) + 1
    y = oracle.spmv(A, x)
    assert np.array_equal(y, [0.0, 1.0 - 8.0 + 3.5, 0.0, 12.0, 0.0])
