"""Pins of the CPU oracle's conjugate-gradient solver.

Checked against numpy.linalg.solve on small systems, against x* = 1 for
b = A*1, against the Krylov bound on the iteration count (from the stencil's
analytic spectrum) and against iteration counts of an independent CG run.
"""
import numpy as np
import pytest

import oracle
from synthetic import CSR, stencil27, stencil27_irregular, uniform_vector


def to_dense(A):
    D = np.zeros((A.n_rows, A.n_cols))
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
    D[rows, A.col] = A.val
    return D


def kappa(grid):
    """Condition number of the 27-point matrix from its analytic eigenvalues."""
    lo, hi = None, None
    ext = []
    for m in grid:
        c = [1 + 2 * np.cos(k * np.pi / (m + 1)) for k in range(1, m + 1)]
        ext.append((min(c), max(c)))
    import itertools

    prods = [np.prod(p) for p in itertools.product(*[(a, b) for a, b in ext])]
    lam = [27.0 - p for p in prods]
    lo, hi = min(lam), max(lam)
    # the extreme eigenvalues come from products of extreme factors
    return hi / lo


@pytest.mark.parametrize("grid", [(3, 4, 5), (6, 5, 4)])
def test_cg_matches_dense_solve(grid):
    A = stencil27(*grid)
    b = uniform_vector(A.n_rows, seed=7)
    x, st, it, rel = oracle.cg(A, b, rtol=1e-13)
    assert st == 0
    xs = np.linalg.solve(to_dense(A), b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-11
    assert oracle.relres(A, b, x) < 1e-12


def test_cg_irregular_matches_dense_solve():
    A = stencil27_irregular(7, 6, 5, seed=2)
    b = uniform_vector(A.n_rows, seed=1)
    x, st, it, rel = oracle.cg(A, b, rtol=1e-13)
    assert st == 0
    xs = np.linalg.solve(to_dense(A), b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-11


@pytest.mark.parametrize("grid,expect", [((16, 16, 16), 27), ((32, 32, 32), 54), ((64, 64, 64), 105)])
def test_cg_ones_solution_iteration_count(grid, expect):
    """b = A*1 -> x* = 1; the iteration count matches an independent CG run within 3."""
    A = stencil27(*grid)
    b = oracle.spmv(A, np.ones(A.n_cols))
    x, st, it, rel = oracle.cg(A, b, rtol=1e-10)
    assert st == 0
    assert abs(it - expect) <= 3
    assert rel <= 1e-10
    assert oracle.relres(A, b, x) <= 2e-10
    assert np.abs(x - 1.0).max() < 1e-7
    # Krylov bound: it <= ceil(0.5 sqrt(kappa) ln(2 / tol))
    assert it <= int(np.ceil(0.5 * np.sqrt(kappa(grid)) * np.log(2 / 1e-10)))


@pytest.mark.parametrize("grid,expect", [((16, 16, 16), 43), ((32, 32, 32), 82)])
def test_cg_random_rhs_iteration_count(grid, expect):
    A = stencil27(*grid)
    b = uniform_vector(A.n_rows, seed=0)
    x, st, it, rel = oracle.cg(A, b, rtol=1e-10)
    assert st == 0 and abs(it - expect) <= 3
    assert oracle.relres(A, b, x) <= 2e-10


def test_kappa_closed_form_values():
    assert abs(kappa((16, 16, 16)) - 39) < 1.0
    assert abs(kappa((104, 104, 104)) - 1489) < 2.0


def test_cg_zero_rhs():
    A = stencil27(4, 4, 4)
    x, st, it, rel = oracle.cg(A, np.zeros(A.n_rows))
    assert st == 0 and it == 0 and np.all(x == 0)


def test_cg_not_spd_reports_breakdown():
    A = stencil27(4, 4, 4)
    A.val[:] = -A.val  # negative definite
    x, st, it, rel = oracle.cg(A, np.ones(A.n_rows))
    assert st == -6 and it == 1


def test_cg_max_iter():
    A = stencil27(16, 16, 16)
    b = uniform_vector(A.n_rows, seed=0)
    x, st, it, rel = oracle.cg(A, b, rtol=1e-10, max_iter=5)
    assert st == -7 and it == 5 and rel > 1e-10


def test_cg_mutation_without_beta_is_detected():
    """A CG that drops the beta term (steepest descent) misses the iteration-count pin."""
    A = stencil27(16, 16, 16)
    b = oracle.spmv(A, np.ones(A.n_cols))
    x = np.zeros(A.n_rows)
    r = b.copy()
    it = 0
    while np.linalg.norm(r) > 1e-10 * np.linalg.norm(b) and it < 200:
        q = oracle.spmv(A, r)
        a = (r @ r) / (r @ q)
        x += a * r
        r -= a * q
        it += 1
    assert abs(it - 27) > 3
