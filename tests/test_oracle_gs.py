"""Pins of the oracle's multicolor symmetric Gauss-Seidel (oracle/gs.py).

* the greedy coloring of a 27-point stencil is the parity coloring
  (x mod 2) + 2 (y mod 2) + 4 (z mod 2) (8 colors; fewer on thin grids);
* one sweep equals the matrix-splitting form of Gauss-Seidel on the
  color-permuted matrix, forward (D + L) x' = b - U x' and backward
  (D + U) x'' = b - L x', solved with dense triangular solves;
* repeated sweeps converge to A^-1 b on the (diagonally dominant) stencil;
* a planted mistake (the backward half dropped) fails the splitting check;
* the preconditioned CG with M = I takes the C oracle's CG iteration count,
  and with SymGS converges in fewer iterations; its preconditioner is the
  dense M = (D + L) D^-1 (D + U) of the color-permuted matrix.
"""
import itertools

import numpy as np
import pytest
from scipy.linalg import solve_triangular

from oracle import gs
from synthetic import CSR, stencil27, stencil27_irregular, uniform_vector


def parity_coloring(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ((x % 2) + 2 * (y % 2) + 4 * (z % 2)).reshape(-1)


def dense(A):
    D = np.zeros((A.n_rows, A.n_cols))
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
    D[rows, A.col] = A.val
    return D


@pytest.mark.parametrize("grid", [(6, 5, 4), (3, 3, 3), (8, 2, 3), (5, 7, 2)])
def test_stencil_coloring_is_the_parity_coloring(grid):
    A = stencil27(*grid)
    c = gs.greedy_coloring(A)
    p = parity_coloring(*grid)
    # the greedy colors are the parity classes, numbered by first appearance
    first = {}
    for cp in p:
        first.setdefault(int(cp), len(first))
    assert np.array_equal(c, np.array([first[int(cp)] for cp in p]))
    assert c.max() + 1 == 2 ** sum(m >= 2 for m in grid)


def test_coloring_is_proper_on_an_irregular_matrix():
    A = stencil27_irregular(9, 8, 7, seed=3)
    c = gs.greedy_coloring(A)
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
    off = A.col != rows
    assert np.all(c[rows[off]] != c[A.col[off]])
    # greedy: every row has each smaller color on a lower-numbered neighbour
    D = dense(A) != 0
    for i in range(0, A.n_rows, 37):
        lower = {int(c[j]) for j in np.flatnonzero(D[i] | D[:, i]) if j < i}
        assert set(range(int(c[i]))) <= lower


def _splitting_sweep(A, b, x, color):
    """Forward then backward Gauss-Seidel on P A P^T by dense triangular solves."""
    perm = np.lexsort((np.arange(A.n_rows), color))  # by color, then by row
    M = dense(A)[np.ix_(perm, perm)]
    bp, xp = b[perm], x[perm]
    DL, U = np.tril(M), np.triu(M, 1)
    DU, L = np.triu(M), np.tril(M, -1)
    x1 = solve_triangular(DL, bp - U @ xp, lower=True)
    x2 = solve_triangular(DU, bp - L @ x1, lower=False)
    out = np.empty_like(x2)
    out[perm] = x2
    return out


@pytest.mark.parametrize("make", [lambda: stencil27(5, 4, 3), lambda: stencil27_irregular(6, 5, 4, seed=1)])
def test_sweep_equals_matrix_splitting(make):
    A = make()
    color = gs.greedy_coloring(A)
    b = uniform_vector(A.n_rows, seed=2)
    x0 = uniform_vector(A.n_rows, seed=3)
    got = gs.symgs(A, b, x0, color)
    ref = _splitting_sweep(A, b, x0, color)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_dropped_backward_half_is_detected():
    """A forward-only sweep (a plausible mistake) does not match the splitting form."""
    A = stencil27(5, 4, 3)
    color = gs.greedy_coloring(A)
    b = uniform_vector(A.n_rows, seed=2)
    x0 = uniform_vector(A.n_rows, seed=3)
    perm = np.lexsort((np.arange(A.n_rows), color))
    M = dense(A)[np.ix_(perm, perm)]
    fwd = solve_triangular(np.tril(M), b[perm] - np.triu(M, 1) @ x0[perm], lower=True)
    out = np.empty_like(fwd)
    out[perm] = fwd
    assert np.max(np.abs(out - _splitting_sweep(A, b, x0, color))) > 1e-6


def test_sweeps_converge_to_the_solution():
    A = stencil27(6, 6, 6)
    color = gs.greedy_coloring(A)
    xs = uniform_vector(A.n_rows, seed=5)
    b = dense(A) @ xs
    x = np.zeros(A.n_rows)
    err0 = np.max(np.abs(x - xs))
    for _ in range(60):
        x = gs.symgs(A, b, x, color)
    assert np.max(np.abs(x - xs)) < 1e-10 * err0


def test_diagonal_and_zero_rhs():
    A = stencil27(4, 4, 4)
    d = gs.diagonal(A)
    assert np.all(d == 26.0)
    color = gs.greedy_coloring(A)
    assert np.array_equal(gs.symgs(A, np.zeros(A.n_rows), np.zeros(A.n_rows), color), np.zeros(A.n_rows))


def test_pcg_identity_preconditioner_is_cg():
    """With M = I the preconditioned iteration is textbook CG: the oracle's C CG
    takes the same number of iterations (within 1, summation orders differ)."""
    import oracle

    A = stencil27(12, 11, 10)
    b = oracle.spmv(A, np.ones(A.n_cols))
    color = gs.greedy_coloring(A)
    x, it, rel = gs.pcg(A, b, color, precondition=False)
    _, _, it_ref, _ = oracle.cg(A, b)
    assert abs(it - it_ref) <= 1 and rel <= 1e-10
    assert np.max(np.abs(x - 1)) < 1e-8


def test_pcg_symgs_converges_faster():
    """SymGS preconditioning: the solution of A x = A*1 to 1e-10, in fewer
    iterations than plain CG, and the preconditioner is the symmetric
    Gauss-Seidel matrix M = (D + L) D^-1 (D + U) of the color-permuted A
    (checked on a small grid by a dense solve)."""
    A = stencil27(12, 11, 10)
    b = dense(A) @ np.ones(A.n_rows)
    color = gs.greedy_coloring(A)
    x, it, rel = gs.pcg(A, b, color)
    _, it_cg, _ = gs.pcg(A, b, color, precondition=False)
    assert rel <= 1e-10 and np.max(np.abs(x - 1)) < 1e-8
    assert it < it_cg
    S = stencil27(4, 3, 3)
    cs = gs.greedy_coloring(S)
    r = uniform_vector(S.n_rows, seed=9)
    perm = np.lexsort((np.arange(S.n_rows), cs))
    Mp = dense(S)[np.ix_(perm, perm)]
    D = np.diag(np.diag(Mp))
    Minv_r = np.linalg.solve((np.tril(Mp) @ np.linalg.inv(D)) @ np.triu(Mp), r[perm])
    z = gs.symgs(S, r, np.zeros(S.n_rows), cs, 1)
    assert np.max(np.abs(z[perm] - Minv_r)) <= 1e-13 * np.max(np.abs(Minv_r))
