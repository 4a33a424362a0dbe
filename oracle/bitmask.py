"""Neighbour-bitmask encoding of a sparse matrix -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
use this module.  It shares no code with the GPU library.

Section V compresses the index array by turning every column index into its
displacement from the diagonal and registering each row's displacement
pattern in a table, so that a row stores only the number of its pattern; it
then suggests compressing that final table further.  This encoding takes the
table to its smallest form for matrices with few distinct displacements (a
stencil, also with couplings removed at random): the table is the single
ascending list D of every displacement the matrix holds, and a row stores
which members of D it has as a bitmask, bit k standing for column row + D[k].
No row needs a table entry of its own, so there are no escape rows however
irregular the rows are.

Readings (listed in the design notes):

* D is ascending; a row's entries in column order are its set bits in
  ascending k.  At most 64 displacements are accepted (a 64-bit mask); the
  mask is 4 bytes wide when D has at most 32 members, else 8.
* Values: when the whole matrix holds at most two distinct values (bitwise
  equality, ordered by IEEE-754 totalOrder) they form the value table V and,
  with two, a second mask per row marks the entries holding V[1].  Otherwise
  no table is kept and every value is stored in the row's column order
  (``raw``), as the raw values of DIT are.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .codec import _bits, total_order_key

MAX_DISPLACEMENTS = 64


@dataclass
class BitmaskEncoding:
    n_rows: int
    n_cols: int
    D: np.ndarray  # int64 [ND], ascending
    mask: np.ndarray  # uint64 [n_rows]: bit k <=> entry at column row + D[k]
    V: np.ndarray  # float64 [K], K <= 2
    vmask: np.ndarray  # uint64 [n_rows] (K == 2): bit k <=> that entry holds V[1]; else None
    raw_ptr: np.ndarray  # int64 [n_rows + 1] (K == 0)
    raw: np.ndarray  # float64, each row's values in column order (K == 0)

    @property
    def K(self) -> int:
        return len(self.V)

    @property
    def mask_bytes(self) -> int:
        return 4 if self.D.size <= 32 else 8


def _row_of(row_ptr):
    return np.repeat(np.arange(row_ptr.size - 1, dtype=np.int64), np.diff(row_ptr))


def encode_bitmask(A) -> BitmaskEncoding:
    """Displacement list D, per-row presence masks, values (table of <= 2, or raw)."""
    rp = np.asarray(A.row_ptr, dtype=np.int64)
    n = A.n_rows
    rows = _row_of(rp)
    cols = np.asarray(A.col, dtype=np.int64)
    val = np.asarray(A.val, dtype=np.float64)
    disp = cols - rows
    D = np.unique(disp)
    if D.size > MAX_DISPLACEMENTS:
        raise ValueError(f"{D.size} distinct displacements; the bitmask holds at most {MAX_DISPLACEMENTS}")
    k = np.searchsorted(D, disp)
    bit = np.left_shift(np.uint64(1), k.astype(np.uint64))
    mask = np.zeros(n, dtype=np.uint64)
    np.bitwise_or.at(mask, rows, bit)
    uniq = np.unique(_bits(val))
    if uniq.size <= 2:
        V = uniq[np.argsort(total_order_key(uniq), kind="stable")].view(np.float64).copy()
        vmask = None
        if V.size == 2:
            vmask = np.zeros(n, dtype=np.uint64)
            hi = _bits(val) == V[1:].view(np.uint64)[0]
            np.bitwise_or.at(vmask, rows[hi], bit[hi])
        return BitmaskEncoding(n, A.n_cols, D, mask, V, vmask, np.zeros(n + 1, dtype=np.int64),
                               np.zeros(0, dtype=np.float64))
    # no table: the values of every row in column order (the CSR order)
    return BitmaskEncoding(n, A.n_cols, D, mask, np.zeros(0, dtype=np.float64), None, rp.copy(), val.copy())


def popcount(m) -> np.ndarray:
    """Set bits of each uint64."""
    m = np.asarray(m, dtype=np.uint64)
    c = np.zeros(m.shape, dtype=np.int64)
    for b in range(64):
        c += ((m >> np.uint64(b)) & np.uint64(1)).astype(np.int64)
    return c


def entries(enc: BitmaskEncoding):
    """(row, column, value) of every stored entry, rows ascending, columns ascending."""
    n = enc.n_rows
    ks = np.arange(enc.D.size, dtype=np.uint64)
    present = ((enc.mask[:, None] >> ks[None, :]) & np.uint64(1)).astype(bool)  # [n, ND]
    rows, kk = np.nonzero(present)  # row-major: per row, k ascending
    cols = rows + enc.D[kk]
    if enc.K == 0:
        vals = enc.raw.copy()
    elif enc.K == 1:
        vals = np.full(rows.size, enc.V[0])
    else:
        hi = ((enc.vmask[rows] >> kk.astype(np.uint64)) & np.uint64(1)).astype(bool)
        vals = np.where(hi, enc.V[1], enc.V[0])
    return rows.astype(np.int64), cols.astype(np.int64), vals


def decode_bitmask(enc: BitmaskEncoding):
    """The CSR matrix back (columns ascending per row)."""
    from synthetic import CSR  # the container type only; no arithmetic

    rows, cols, vals = entries(enc)
    rp = np.zeros(enc.n_rows + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=enc.n_rows), out=rp[1:])
    return CSR(enc.n_rows, enc.n_cols, rp, cols.astype(np.int32), vals)


def stream_bytes(enc: BitmaskEncoding) -> dict:
    """Bytes of the encoding: masks per row, values, the displacement list."""
    n = enc.n_rows
    rows = enc.mask_bytes * n * (2 if enc.K == 2 else 1)
    return {"rows": rows, "raw": 8 * int(enc.raw.size), "table": 4 * int(enc.D.size) + 8 * enc.K,
            "total": rows + 8 * int(enc.raw.size) + 4 * int(enc.D.size) + 8 * enc.K}
