"""Symmetric Gauss-Seidel over a multicolor ordering -- TEST INFRASTRUCTURE ONLY.

Only the test-suite and the benchmark's CPU-baseline leg may use this module.
It shares no code with the GPU library.

SymGS is the other kernel that dominates the HPCG iteration the paper
accelerates (Section III, Table I: SymGS beside SpMV); it walks the same
matrix rows.  A sweep updates x_i = (b_i - sum_{j != i} a_ij x_j) / a_ii row
by row, forward through the rows and then backward.  For a GPU the rows are
taken in a multicolor order: rows of one color share no entry, so they can
be updated together, and the sweep visits the colors forward then backward.
The coloring is greedy in row order over the pattern of A + A^T: each row
takes the smallest color that no lower-numbered neighbour holds.

Pins (tests/test_oracle_gs.py): the coloring of a 27-point stencil equals the
parity coloring (x mod 2) + 2 (y mod 2) + 4 (z mod 2); a sweep equals the
matrix-splitting form (D + L) x' = b - U x, (D + U) x'' = b - L x' of the
color-permuted matrix, solved by dense triangular solves; repeated sweeps
converge to A^-1 b on a diagonally dominant matrix; ``pcg`` with M = I
takes the C oracle's CG iteration count, and its SymGS preconditioner equals
the dense M = (D + L) D^-1 (D + U) of the color-permuted matrix; the V-cycle
equals its operator form B_l = S + (I - S A)(S + P B_{l+1} R (I - A S)) built
from dense matrices (S the sweep from zero, R the injection, P = R^T), is
symmetric positive definite, reduces to one sweep on a single level, and
cuts the CG iteration count below the single sweep's.
"""
from __future__ import annotations

import numpy as np


def greedy_coloring(A) -> np.ndarray:
    """Color of every row: greedy in row order over the pattern of A + A^T.

    Plain Python loops: for matrices of a few ten thousand rows at most.
    """
    n = A.n_rows
    rp = np.asarray(A.row_ptr, dtype=np.int64)
    col = np.asarray(A.col, dtype=np.int64)
    nbr = [set() for _ in range(n)]
    for i in range(n):
        for k in range(int(rp[i]), int(rp[i + 1])):
            j = int(col[k])
            if j != i and j < n:
                nbr[i].add(j)
                nbr[j].add(i)
    color = np.full(n, -1, dtype=np.int64)
    for i in range(n):
        used = {int(color[j]) for j in nbr[i] if j < i}
        c = 0
        while c in used:
            c += 1
        color[i] = c
    return color


def diagonal(A) -> np.ndarray:
    """a_ii of every row (0 where the row holds no diagonal entry)."""
    rows = np.repeat(np.arange(A.n_rows, dtype=np.int64), np.diff(A.row_ptr))
    d = np.zeros(A.n_rows, dtype=np.float64)
    on = np.asarray(A.col, dtype=np.int64) == rows
    d[rows[on]] = np.asarray(A.val)[on]
    return d


def symgs(A, b, x, color, sweeps: int = 1, reverse: bool = False) -> np.ndarray:
    """`sweeps` symmetric Gauss-Seidel sweeps on A x = b in the order of `color`.

    Each sweep visits the colors 0, 1, ..., C-1 and then C-1, ..., 0 (with
    reverse=True: C-1, ..., 0 and then 0, ..., C-1); the rows
    of a color are updated with x_i = (b_i - sum_{j != i} a_ij x_j) / a_ii,
    every off-diagonal product taken from the current x.  Returns the new x.
    """
    n = A.n_rows
    x = np.array(x, dtype=np.float64, copy=True)
    b = np.asarray(b, dtype=np.float64)
    color = np.asarray(color, dtype=np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(A.row_ptr))
    col = np.asarray(A.col, dtype=np.int64)
    val = np.asarray(A.val, dtype=np.float64)
    d = diagonal(A)
    off = col != rows
    n_colors = int(color.max()) + 1 if n else 0
    rows_of = [np.flatnonzero(color == c) for c in range(n_colors)]
    ent_of = [np.flatnonzero(off & (color[rows] == c)) for c in range(n_colors)]
    up, down = list(range(n_colors)), list(range(n_colors - 1, -1, -1))
    order = down + up if reverse else up + down
    for _ in range(sweeps):
        for c in order:
            R, e = rows_of[c], ent_of[c]
            s = np.bincount(rows[e], weights=val[e] * x[col[e]], minlength=n)
            x[R] = (b[R] - s[R]) / d[R]
    return x


def _matvec(A, v):
    rows = np.repeat(np.arange(A.n_rows, dtype=np.int64), np.diff(A.row_ptr))
    return np.bincount(rows, weights=np.asarray(A.val) * v[np.asarray(A.col)], minlength=A.n_rows)


def pcg(A, b, color, rtol: float = 1e-10, max_iter: int = 100000, precondition: bool = True):
    """Preconditioned CG from x0 = 0, with M^-1 r = one symmetric Gauss-Seidel
    sweep on A z = r from z = 0 in the multicolor order `color` (the role
    SymGS plays inside the preconditioner of the HPCG iteration, Table I).
    With precondition=False, M = I (plain CG).  Stops when ||r|| <= rtol ||b||.
    Returns (x, iterations, ||r|| / ||b||)."""
    n = A.n_rows

    def prec(r):
        return symgs(A, r, np.zeros(n), color, 1) if precondition else r.copy()

    return _pcg(A, b, prec, rtol, max_iter)


def vcycle(levels, f2c, colors, r, level: int = 0) -> np.ndarray:
    """One V-cycle of the geometric multigrid preconditioner, z ~ A_l^-1 r, in
    the order of Table I (Section III): on every level but the coarsest, z = 0,
    one SymGS sweep, the residual r - A z by SpMV, restriction by injection
    (r_c[i] = (r - A z)[f2c[i]]), the V-cycle on the next level, prolongation
    by injection (z[f2c[i]] += z_c[i]) and one more SymGS sweep; on the
    coarsest level, z = 0 and one SymGS sweep.  levels[l]: CSR of level l;
    f2c[l]: fine row of level l for each row of level l + 1; colors[l]: the
    multicolor order of level l.

    The smoother visits the colors in reverse (C-1 down to 0, then back up).
    A Gauss-Seidel update leaves zero residual on the rows it updates, and
    the rows updated last keep it; in the forward order those are color 0,
    which on the stencil hierarchy holds exactly the injection points (row 0
    starts the greedy coloring), so the restricted residual would vanish and
    the coarse levels would contribute nothing."""
    A = levels[level]
    z = symgs(A, r, np.zeros(A.n_rows), colors[level], 1, reverse=True)
    if level + 1 == len(levels):
        return z
    m = np.asarray(f2c[level], dtype=np.int64)
    rc = (np.asarray(r, dtype=np.float64) - _matvec(A, z))[m]
    zc = vcycle(levels, f2c, colors, rc, level + 1)
    z[m] += zc
    return symgs(A, r, z, colors[level], 1, reverse=True)


def pcg_mg(levels, f2c, colors, b, rtol: float = 1e-10, max_iter: int = 100000):
    """CG on levels[0] x = b preconditioned by one V-cycle per iteration (the
    HPCG iteration of Table I).  Returns (x, iterations, ||r|| / ||b||)."""
    return _pcg(levels[0], b, lambda r: vcycle(levels, f2c, colors, r), rtol, max_iter)


def _pcg(A, b, prec, rtol, max_iter):
    """Textbook preconditioned CG (Saad, Alg. 9.1) from x0 = 0."""
    b = np.asarray(b, dtype=np.float64)
    n = A.n_rows
    x = np.zeros(n)
    r = b.copy()
    bn = np.sqrt(b @ b)
    if bn == 0.0:
        return x, 0, 0.0
    z = prec(r)
    p = z.copy()
    rz = r @ z
    it = 0
    while it < max_iter:
        q = _matvec(A, p)
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        rn = np.sqrt(r @ r)
        if rn <= rtol * bn:
            break
        z = prec(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, float(np.sqrt(r @ r) / bn)
