"""Pins of the oracle's neighbour-bitmask encoding (CPU only).

The encoding is lossless, so its pins are the definition itself: a
hand-worked example, the 27-point stencil's closed form (its displacement list
and which neighbours each row has follow from the grid coordinates), the
lossless round trip, and the value-table rule.
"""
import numpy as np
import pytest

import oracle
from oracle import bitmask as bm
from synthetic import CSR, stencil27, stencil27_irregular, uniform_vector


def test_hand_worked_tridiagonal():
    """4 x 4 matrix tridiag(-1, 2, -1): D = [-1, 0, 1]; row 0 holds d = 0, 1
    (bits 1, 2 -> 0b110), rows 1-2 all three (0b111), row 3 d = -1, 0 (0b011);
    V = [-1, 2] and the V[1] bit is the diagonal's (0b010) in every row."""
    rp = np.array([0, 2, 5, 8, 10])
    col = np.array([0, 1, 0, 1, 2, 1, 2, 3, 2, 3], dtype=np.int32)
    val = np.array([2, -1, -1, 2, -1, -1, 2, -1, -1, 2], dtype=np.float64)
    A = CSR(4, 4, rp, col, val)
    enc = bm.encode_bitmask(A)
    assert enc.D.tolist() == [-1, 0, 1]
    assert enc.mask.tolist() == [0b110, 0b111, 0b111, 0b011]
    assert enc.V.tolist() == [-1.0, 2.0] and enc.K == 2
    assert enc.vmask.tolist() == [0b010] * 4
    assert enc.mask_bytes == 4
    assert bm.stream_bytes(enc) == {"rows": 32, "raw": 0, "table": 28, "total": 60}


def _stencil_closed_form(nx, ny, nz):
    """Displacements and per-row neighbour sets of the 27-point stencil from the
    coordinates alone (rows x-fastest)."""
    offs = sorted({dz * nx * ny + dy * nx + dx for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                   if (nx > 1 or dx == 0) and (ny > 1 or dy == 0) and (nz > 1 or dz == 0)})
    i = np.arange(nx * ny * nz)
    ix, iy, iz = i % nx, (i // nx) % ny, i // (nx * ny)
    mask = np.zeros(i.size, dtype=np.uint64)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                ok = (ix + dx >= 0) & (ix + dx < nx) & (iy + dy >= 0) & (iy + dy < ny) & (iz + dz >= 0) & (iz + dz < nz)
                d = dz * nx * ny + dy * nx + dx
                if d in offs:
                    mask[ok] |= np.uint64(1) << np.uint64(offs.index(d))
    return np.array(offs), mask


@pytest.mark.parametrize("grid", [(16, 16, 16), (7, 5, 3), (9, 1, 4), (1, 1, 5)])
def test_stencil_closed_form(grid):
    A = stencil27(*grid)
    enc = bm.encode_bitmask(A)
    D, mask = _stencil_closed_form(*grid)
    assert np.array_equal(enc.D, D)
    assert np.array_equal(enc.mask, mask)
    assert np.array_equal(bm.popcount(enc.mask), np.diff(A.row_ptr))
    # V = {-1, 26}; only the diagonal (d = 0) holds 26
    assert enc.V.tolist() == [-1.0, 26.0]
    d0 = np.uint64(1) << np.uint64(int(np.flatnonzero(D == 0)[0]))
    assert np.all(enc.vmask == d0)


@pytest.mark.parametrize("make", [lambda: stencil27(16, 16, 16), lambda: stencil27_irregular(20, 17, 13, seed=1),
                                  lambda: stencil27(5, 3, 4)])
def test_round_trip_and_spmv(make):
    A = make()
    enc = bm.encode_bitmask(A)
    B = bm.decode_bitmask(enc)
    assert np.array_equal(B.row_ptr, A.row_ptr) and np.array_equal(B.col, A.col)
    assert np.array_equal(B.val.view(np.uint64), np.asarray(A.val).view(np.uint64))
    x = uniform_vector(A.n_cols, seed=2)
    rows, cols, vals = bm.entries(enc)
    y = np.zeros(A.n_rows)
    np.add.at(y, rows, vals * x[cols])
    yref = oracle.spmv(A, x)
    scale = oracle.spmv(CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, np.abs(A.val)), np.abs(x))
    assert np.all(np.abs(y - yref) <= 1e-14 * scale)


def test_irregular_values_are_raw_in_column_order():
    """The irregular stencil's values are all distinct: no table, every value
    stored in the row's column order; its displacements are a subset of the
    full stencil's and each row's mask a subset of the full row's."""
    A = stencil27_irregular(20, 17, 13, seed=1)
    enc = bm.encode_bitmask(A)
    assert enc.K == 0 and enc.vmask is None
    assert np.array_equal(enc.raw_ptr, A.row_ptr) and np.array_equal(enc.raw, A.val)
    D, mask = _stencil_closed_form(20, 17, 13)
    assert set(enc.D.tolist()) <= set(D.tolist())
    full = np.zeros(A.n_rows, dtype=np.uint64)
    pos = {d: k for k, d in enumerate(D.tolist())}
    for k, d in enumerate(enc.D.tolist()):
        has = ((enc.mask >> np.uint64(k)) & np.uint64(1)).astype(bool)
        full[has] |= np.uint64(1) << np.uint64(pos[d])
    assert np.all((full & ~mask) == 0)
    assert np.array_equal(bm.popcount(enc.mask), np.diff(A.row_ptr))
    assert bm.stream_bytes(enc)["raw"] == 8 * A.nnz


def test_value_table_rule():
    """One distinct value: K = 1, no second mask; three: no table; -0.0 and
    +0.0 are different values (bitwise equality)."""
    A = stencil27(6, 5, 4)
    A.val[:] = 3.0
    enc = bm.encode_bitmask(A)
    assert enc.K == 1 and enc.vmask is None and enc.V.tolist() == [3.0]
    A.val[0] = 1.5
    A.val[1] = 2.5
    enc = bm.encode_bitmask(A)
    assert enc.K == 0 and np.array_equal(enc.raw, A.val)
    A.val[:] = 0.0
    A.val[::2] = -0.0
    enc = bm.encode_bitmask(A)
    assert enc.K == 2 and np.signbit(enc.V[0]) and not np.signbit(enc.V[1])
    B = bm.decode_bitmask(enc)
    assert np.array_equal(B.val.view(np.uint64), A.val.view(np.uint64))


def test_limits():
    """65 distinct displacements do not fit a 64-bit mask; 33 need the 8-byte width;
    empty rows have an empty mask."""
    n = 80
    cols = np.arange(65, dtype=np.int32)
    A = CSR(n, n, np.concatenate([[0], np.full(n, 65)]), cols, np.ones(65))
    with pytest.raises(ValueError):
        bm.encode_bitmask(A)
    A = CSR(n, n, np.concatenate([[0], np.full(n, 33)]), cols[:33], np.ones(33))
    enc = bm.encode_bitmask(A)
    assert enc.D.size == 33 and enc.mask_bytes == 8
    assert enc.mask[0] == (1 << 33) - 1 and np.all(enc.mask[1:] == 0)
