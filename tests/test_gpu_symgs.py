"""GPU multicolor symmetric Gauss-Seidel against the oracle (oracle/gs.py), through the C ABI.

* the coloring equals the oracle's greedy row-order coloring exactly, and on
  the full 104^3 stencil the parity coloring (x mod 2) + 2 (y mod 2) + 4 (z mod 2);
* sweeps equal the oracle's to a tolerance from the arithmetic: each row
  update is a <= 27-term sum with relative error <= gamma_27 of
  (|b_i| + sum |a_ij||x_j|) / |a_ii| <= about 1.5e-15 on these matrices, and
  a sweep chains 16 color steps of a diagonally dominant (contracting)
  iteration, so 1e-12 of the vectors' size leaves a wide margin;
* DITV gives DIT's result bit for bit (same entries in the same order);
* one-sided patterns (neighbours only through A^T) and more than 64 colors
  (the coloring's general path) give the oracle's colors and sweeps;
* bad inputs are rejected (non-square, zero diagonal, negative sweeps).
"""
import sys

import numpy as np
import pytest

from oracle import gs
from synthetic import CSR, stencil27, stencil27_irregular, uniform_vector

from gpu_util import compress, lib, torch_mod

pytestmark = pytest.mark.gpu

FORMATS = ["ELL", "DT", "DIT", "DITV"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def parity_coloring(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ((x % 2) + 2 * (y % 2) + 4 * (z % 2)).reshape(-1)


def run(M, b, x0, sweeps=1):
    torch = torch_mod()
    x = torch.from_numpy(np.array(x0)).cuda()
    M.symgs(torch.from_numpy(np.asarray(b)).cuda(), x, sweeps=sweeps)
    torch.cuda.synchronize()
    return x.cpu().numpy()


def close(got, ref, *vecs):
    scale = max([1.0] + [float(np.max(np.abs(v))) for v in (ref,) + vecs])
    return float(np.max(np.abs(got - ref))) <= 1e-12 * scale


@pytest.mark.parametrize("make", [lambda: stencil27(12, 10, 9), lambda: stencil27_irregular(10, 9, 8, seed=3),
                                  lambda: stencil27(7, 1, 5)])
def test_coloring_equals_oracle(make):
    say("case: symgs coloring")
    A = make()
    M = compress(A, fmt="DIT")
    nc, col = M.colors()
    ref = gs.greedy_coloring(A)
    assert nc == int(ref.max()) + 1
    assert np.array_equal(col.cpu().numpy().astype(np.int64), ref)


def _csr(n, rows):
    """CSR from per-row {column: value} dicts (columns sorted)."""
    rp, cols, vals = [0], [], []
    for r in rows:
        for j in sorted(r):
            cols.append(j)
            vals.append(r[j])
        rp.append(len(cols))
    return CSR(n, n, np.array(rp, dtype=np.int64), np.array(cols, dtype=np.int32), np.array(vals))


def _asymmetric(n=400, block=0):
    """Tridiagonal rows plus one-sided long-range entries (row i holds column
    i + 5 + i % 11 for i % 3 == 0, not the reverse), so that some rows' only
    lower-numbered neighbours come through A^T; with block = k, rows 100 ..
    100 + k - 1 also form a fully coupled block, which needs k colors."""
    rows = [dict() for _ in range(n)]
    for i in range(n):
        rows[i][i] = 4.0
        for j in (i - 1, i + 1):
            if 0 <= j < n:
                rows[i][j] = -1.0
        if i % 3 == 0 and i + 5 + i % 11 < n:
            rows[i][i + 5 + i % 11] = -0.5
    for i in range(100, 100 + block):
        for j in range(100, 100 + block):
            if j != i:
                rows[i][j] = -1.0
        rows[i][i] = 2.0 * block
    return _csr(n, rows)


@pytest.mark.parametrize("block,fmt", [(0, "DIT"), (0, "ELL"), (70, "ELL")])
def test_coloring_asymmetric_and_over_64_colors(block, fmt):
    """One-sided entries (neighbours only through A^T) and, with a fully
    coupled block of 70 rows, more than 64 colors (the coloring then takes its
    general path): the colors equal the oracle's greedy coloring and a sweep
    equals the oracle's."""
    say("case: symgs coloring asymmetric", block, fmt)
    A = _asymmetric(block=block)
    M = compress(A, fmt=fmt)
    nc, col = M.colors()
    ref = gs.greedy_coloring(A)
    assert nc == int(ref.max()) + 1 and (nc >= 70 if block else nc < 64)
    assert np.array_equal(col.cpu().numpy().astype(np.int64), ref)
    b = uniform_vector(A.n_rows, seed=6)
    x0 = uniform_vector(A.n_rows, seed=7)
    assert close(run(M, b, x0, 1), gs.symgs(A, b, x0, ref, 1), b, x0)


@pytest.mark.parametrize("fmt", FORMATS)
@pytest.mark.parametrize("make", [lambda: stencil27(12, 10, 9), lambda: stencil27_irregular(14, 12, 10, seed=1)])
def test_sweeps_equal_oracle(fmt, make):
    say("case: symgs sweeps", fmt)
    A = make()
    M = compress(A, fmt=fmt)
    color = gs.greedy_coloring(A)
    b = uniform_vector(A.n_rows, seed=4)
    x0 = uniform_vector(A.n_rows, seed=5)
    for sweeps in (1, 3):
        got = run(M, b, x0, sweeps)
        ref = gs.symgs(A, b, x0, color, sweeps)
        assert close(got, ref, b, x0)
    assert np.array_equal(run(M, b, x0, 0), x0)  # no sweep: x untouched


def test_full_size_104():
    """The 104^3 stencil: the parity coloring, and one sweep from x = 0 equal
    to the oracle's (the same launch the benchmark times)."""
    say("case: symgs 104^3")
    A = stencil27(104, 104, 104)
    M = compress(A, fmt="DIT")
    nc, col = M.colors()
    assert nc == 8 and np.array_equal(col.cpu().numpy(), parity_coloring(104, 104, 104))
    b = uniform_vector(A.n_rows, seed=6)
    x0 = np.zeros(A.n_rows)
    got = run(M, b, x0)
    ref = gs.symgs(A, b, x0, parity_coloring(104, 104, 104))
    assert close(got, ref, b)


def test_ditv_equals_dit():
    say("case: symgs DITV vs DIT")
    A = stencil27(20, 18, 16)
    b = uniform_vector(A.n_rows, seed=7)
    x0 = uniform_vector(A.n_rows, seed=8)
    assert np.array_equal(run(compress(A, fmt="DITV"), b, x0, 2), run(compress(A, fmt="DIT"), b, x0, 2))


def test_bad_inputs_are_rejected():
    say("case: symgs errors")
    torch = torch_mod()
    P = lib()
    # a row without its diagonal entry
    A = stencil27(4, 4, 4)
    keep = np.ones(A.nnz, dtype=bool)
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
    keep[np.flatnonzero((rows == 5) & (A.col == 5))] = False
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows[keep], minlength=A.n_rows))])
    B = CSR(A.n_rows, A.n_cols, rp, A.col[keep], A.val[keep])
    M = compress(B, fmt="DIT")
    z = torch.zeros(B.n_rows, dtype=torch.float64, device="cuda")
    with pytest.raises(P.SpmvcError):
        M.symgs(z, z.clone())
    # a non-square matrix
    C = CSR(2, 3, np.array([0, 2, 3]), np.array([0, 2, 1], dtype=np.int32), np.array([1.0, 2.0, 3.0]))
    Mc = compress(C, fmt="DIT")
    with pytest.raises(P.SpmvcError):
        Mc.symgs(torch.zeros(2, dtype=torch.float64, device="cuda"))
    # negative sweeps
    M2 = compress(A, fmt="DIT")
    with pytest.raises(P.SpmvcError):
        M2.symgs(z, z.clone(), sweeps=-1)


@pytest.mark.parametrize("fmt", FORMATS + ["BMASK"])
@pytest.mark.parametrize("make", [lambda: stencil27(12, 10, 9), lambda: stencil27_irregular(10, 9, 8, seed=3)])
def test_color_order(make, fmt):
    """spmv_color_order: B = P A P^T with P the rows color by color -- the
    oracle's greedy coloring sorted stably by color -- equal entry for entry
    to the oracle's permutation of A; B's coloring is the induced one (color
    ranges); sweeps on B with b[perm], x0[perm] give the oracle's sweep on A,
    permuted."""
    say("case: color order", fmt)
    from oracle import reorder

    torch = torch_mod()
    P = lib()
    A = make()
    M = compress(A, fmt=fmt)
    try:
        B, perm = M.color_order()
    except P.SpmvcError as e:  # BMASK: the reordered matrix has more than 64 displacements
        assert fmt == "BMASK" and e.status == -8
        return
    color = gs.greedy_coloring(A)
    ref_perm = np.argsort(color, kind="stable")
    perm = perm.cpu().numpy().astype(np.int64)
    assert np.array_equal(perm, ref_perm)
    R = reorder.permute(A, perm)
    rp, col, val = B.decompress()
    assert np.array_equal(rp.cpu().numpy(), R.row_ptr) and np.array_equal(col.cpu().numpy(), R.col)
    assert np.array_equal(val.cpu().numpy().view(np.uint64), np.asarray(R.val).view(np.uint64))
    nc, bcol = B.colors()
    assert nc == int(color.max()) + 1
    assert np.array_equal(bcol.cpu().numpy().astype(np.int64), color[perm])
    b = uniform_vector(A.n_rows, seed=5)
    x0 = uniform_vector(A.n_rows, seed=6)
    ref = gs.symgs(A, b, x0, color, sweeps=2)
    got = run(B, b[perm], x0[perm], sweeps=2)
    assert close(got, ref[perm], b, x0)


def test_color_order_full_size_104():
    """The 104^3 stencil's color-ordered twin: 8 colors of 140,608 rows, the
    permutation of the parity coloring, and a sweep equal to the oracle's."""
    say("case: color order 104^3")
    A = stencil27(104, 104, 104)
    M = compress(A, fmt="DIT")
    B, perm = M.color_order()
    color = parity_coloring(104, 104, 104)
    perm = perm.cpu().numpy().astype(np.int64)
    assert np.array_equal(perm, np.argsort(color, kind="stable"))
    b = uniform_vector(A.n_rows, seed=7)
    x0 = np.zeros(A.n_rows)
    ref = gs.symgs(A, b, x0, color, sweeps=1)
    got = run(B, b[perm], x0[perm], sweeps=1)
    assert close(got, ref[perm], b)
