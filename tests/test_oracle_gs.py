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


def _sweep_operator(A, color):
    """Dense S = M^-1, M = (D + L) D^-1 (D + U) of the color-permuted A, in the
    original row order: one SymGS sweep from zero maps r to S r."""
    perm = np.lexsort((np.arange(A.n_rows), color))
    Mp = dense(A)[np.ix_(perm, perm)]
    D = np.diag(np.diag(Mp))
    Sp = np.linalg.inv((np.tril(Mp) @ np.linalg.inv(D)) @ np.triu(Mp))
    S = np.empty_like(Sp)
    S[np.ix_(perm, perm)] = Sp
    return S


def _vcycle_operator(levels, f2c, colors, level=0, post=True):
    """B_l = S + (I - S A)(S + P B_{l+1} R (I - A S)) from dense matrices, with
    R the injection (R[i, f2c[i]] = 1) and P = R^T; B_last = S."""
    A = dense(levels[level])
    S = _sweep_operator(levels[level], colors[level].max() - colors[level])  # smoother in reverse color order
    if level + 1 == len(levels):
        return S
    n = A.shape[0]
    R = np.zeros((levels[level + 1].n_rows, n))
    R[np.arange(R.shape[0]), f2c[level]] = 1.0
    Bc = _vcycle_operator(levels, f2c, colors, level + 1, post)
    z2 = S + R.T @ Bc @ R @ (np.eye(n) - A @ S)
    return S + (np.eye(n) - S @ A) @ z2 if post else z2


def test_hierarchy_injects_the_even_points():
    from synthetic import stencil_hierarchy

    mats, f2c = stencil_hierarchy(8, 12, 4, 3)
    assert [m.grid for m in mats] == [(8, 12, 4), (4, 6, 2), (2, 3, 1)]
    assert [len(m) for m in f2c] == [48, 6]
    for lev, m in enumerate(f2c):
        nx, ny, nz = mats[lev].grid
        i = np.arange(mats[lev].n_rows)
        even = np.flatnonzero(((i % nx) % 2 == 0) & (((i // nx) % ny) % 2 == 0) & ((i // (nx * ny)) % 2 == 0))
        assert np.array_equal(np.asarray(m, dtype=np.int64), even)
    with pytest.raises(ValueError):
        stencil_hierarchy(6, 6, 6, 3)


def test_vcycle_equals_operator_form_and_is_spd():
    """The oracle's V-cycle, applied to the unit vectors, is the dense operator
    B_0 of a 3-level hierarchy; B_0 is symmetric positive definite, while the
    V-cycle without post-smoothing (a plausible mistake) is not symmetric."""
    from synthetic import stencil_hierarchy

    mats, f2c = stencil_hierarchy(8, 8, 4, 3)
    colors = [gs.greedy_coloring(m) for m in mats]
    n = mats[0].n_rows
    got = np.column_stack([gs.vcycle(mats, f2c, colors, e) for e in np.eye(n)])
    ref = _vcycle_operator(mats, f2c, colors)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert np.max(np.abs(got - got.T)) <= 1e-12 * np.max(np.abs(got))
    assert np.linalg.eigvalsh(0.5 * (got + got.T)).min() > 0
    pre_only = _vcycle_operator(mats, f2c, colors, post=False)
    assert np.max(np.abs(pre_only - pre_only.T)) > 1e-3 * np.max(np.abs(pre_only))


def test_single_level_vcycle_is_one_sweep():
    """With one level the V-cycle is z = 0 plus one sweep in reverse color
    order: MG-preconditioned CG is then the SymGS-preconditioned CG with the
    colors renumbered C-1-c, iterate for iterate."""
    A = stencil27(9, 8, 7)
    b = dense(A) @ np.ones(A.n_rows)
    c = gs.greedy_coloring(A)
    x1, it1, rel1 = gs.pcg_mg([A], [], [c], b)
    x2, it2, rel2 = gs.pcg(A, b, c.max() - c)
    assert it1 == it2 and rel1 == rel2 and np.array_equal(x1, x2)


def test_mg_pcg_converges_faster_than_one_sweep():
    from synthetic import stencil_hierarchy

    mats, f2c = stencil_hierarchy(16, 16, 16, 4)
    colors = [gs.greedy_coloring(m) for m in mats]
    A = mats[0]
    b = dense(A) @ np.ones(A.n_rows)
    x, it, rel = gs.pcg_mg(mats, f2c, colors, b)
    _, it_gs, _ = gs.pcg(A, b, colors[0])
    assert rel <= 1e-10 and np.max(np.abs(x - 1)) < 1e-8
    assert it < it_gs


def test_forward_order_smoother_zeroes_the_injected_residual():
    """Why the V-cycle's smoother runs the colors in reverse: after a sweep in
    the forward order the residual vanishes on color 0, which on the stencil
    hierarchy is exactly the set of injection points; in reverse order it
    does not."""
    from synthetic import stencil_hierarchy

    mats, f2c = stencil_hierarchy(8, 8, 8, 2)
    A, c = mats[0], gs.greedy_coloring(mats[0])
    assert set(np.flatnonzero(c == 0)) == set(f2c[0].tolist())
    r = uniform_vector(A.n_rows, seed=4)
    res = lambda z: (r - dense(A) @ z)[f2c[0]]
    assert np.abs(res(gs.symgs(A, r, np.zeros(A.n_rows), c))).max() < 1e-13
    assert np.abs(res(gs.symgs(A, r, np.zeros(A.n_rows), c, reverse=True))).max() > 0.1
