"""Two-sided pins of the oracle's true relative residual ||b - A x||_2 / ||b||_2.

Every CG, mixed-precision, batched, preconditioned and multigrid parity test
accepts a GPU solve by this one function, so it is pinned here to values
that follow from the definition and the stencil's structure alone, computed
without the oracle:

* x = 0 gives r = b, so the result is exactly 1 for any b != 0;
* b = A*1 and x = 1 + delta*e_k give b - A x = -delta * (column k of A), so
  the result is delta * ||A e_k|| / ||A*1||.  Column k of the 27-point
  stencil holds 26 and one -1 per neighbour of grid point k, and (A*1)_i is
  26 minus the neighbour count of point i; both are counted here from the
  grid coordinates.  With delta a power of two every product and sum in the
  residual is exact, so the only rounding is in the two square roots and
  the division: the comparison is to a few ulps.  A missing square root, a
  missing division by ||b||, a dropped sign or a transposed operand each
  changes the value by orders of magnitude or by the column/row norm ratio;
* with b = 0 the function reports ||A x|| itself (the documented fallback);
* scaling b and x by the same power of two leaves the result unchanged.
"""
import numpy as np
import pytest

import oracle
from synthetic import stencil27, stencil27_irregular, uniform_vector


def neighbour_counts(nx, ny, nz):
    """Neighbours (excluding the point) of every grid point, x-fastest numbering."""
    def span(m):
        i = np.arange(m)
        return np.minimum(i + 1, m - 1) - np.maximum(i - 1, 0) + 1

    sx, sy, sz = span(nx), span(ny), span(nz)
    cnt = sz[:, None, None] * sy[None, :, None] * sx[None, None, :]
    return (cnt - 1).reshape(-1).astype(np.float64)


def test_zero_iterate_gives_one():
    A = stencil27(7, 6, 5)
    for seed in (0, 1, 2):
        b = uniform_vector(A.n_rows, seed=seed)
        assert oracle.relres(A, b, np.zeros(A.n_rows)) == 1.0


@pytest.mark.parametrize("grid", [(8, 8, 8), (13, 7, 5)])
@pytest.mark.parametrize("kind", ["interior", "face", "corner"])
@pytest.mark.parametrize("delta_exp", [-20, -33])
def test_unit_perturbation_closed_form(grid, kind, delta_exp):
    nx, ny, nz = grid
    A = stencil27(nx, ny, nz)
    nb = neighbour_counts(nx, ny, nz)
    ax1 = 26.0 - nb  # (A*1)_i
    if kind == "interior":
        k = (nx // 2) + nx * ((ny // 2) + ny * (nz // 2))
    elif kind == "face":
        k = (nx // 2) + nx * (ny // 2)  # z = 0 face
    else:
        k = 0
    delta = 2.0 ** delta_exp
    b = 26.0 - nb  # A*1 from the closed form, not from the oracle's SpMV
    x = np.ones(A.n_rows)
    x[k] += delta
    # column k: 26 on the diagonal, -1 for each neighbour of point k
    col_norm = np.sqrt(26.0 ** 2 + nb[k])
    expect = delta * col_norm / np.sqrt(np.sum(ax1 * ax1))
    got = oracle.relres(A, b, x)
    assert got == pytest.approx(expect, rel=4e-16 * 8)
    # the readings a slip in the oracle would give are far away
    assert abs(got - delta * col_norm) > 1e-3 * expect
    assert abs(got - expect ** 2) > 1e-3 * expect


def test_zero_rhs_reports_absolute_residual():
    A = stencil27(5, 5, 5)
    x = np.zeros(A.n_rows)
    x[62] = 0.5  # centre point: 26 neighbours
    expect = 0.5 * np.sqrt(26.0 ** 2 + 26.0)
    assert oracle.relres(A, np.zeros(A.n_rows), x) == pytest.approx(expect, rel=1e-15)


def test_scale_invariance_by_powers_of_two():
    A = stencil27_irregular(9, 8, 7, seed=3)
    b = uniform_vector(A.n_rows, seed=4)
    x = uniform_vector(A.n_rows, seed=5)
    r0 = oracle.relres(A, b, x)
    for e in (-40, 17):
        c = 2.0 ** e
        assert oracle.relres(A, c * b, c * x) == r0


def test_matches_dense_definition_on_irregular_matrix():
    """Against numpy's own norm of the dense residual (a library routine for
    each step: dense product, vector 2-norm)."""
    A = stencil27_irregular(6, 5, 4, seed=1)
    D = np.zeros((A.n_rows, A.n_cols))
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
    D[rows, A.col] = A.val
    b = uniform_vector(A.n_rows, seed=8)
    x = uniform_vector(A.n_rows, seed=9)
    expect = np.linalg.norm(b - D @ x) / np.linalg.norm(b)
    assert oracle.relres(A, b, x) == pytest.approx(expect, rel=1e-13)
