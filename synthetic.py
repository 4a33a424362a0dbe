"""Seeded synthetic inputs: 27-point stencil matrices in CSR form, vectors.

This module only *generates inputs*.  It holds none of the compression,
SpMV or CG arithmetic, and it is shared by the CPU oracle's tests and the
GPU path's tests/benchmark so that both consume identical CSR arrays.

Matrix families (the paper's workload is the HPCG matrix: a 3-D diffusion
problem discretised with a 27-point stencil on a regular grid, diagonal 26,
each existing neighbour -1; Section III-A, "The HPCG benchmark"):

* ``stencil27(nx, ny, nz)`` - the HPCG matrix on one nx*ny*nz grid,
  truncated at the grid faces.  Rows are numbered x-fastest:
  ``row = ix + nx*(iy + ny*iz)``.  Columns within a row are ascending.
* ``stencil27_irregular(nx, ny, nz, seed, p_remove)`` - the same stencil with
  a seeded, symmetric removal of off-diagonal couplings and random
  off-diagonal values, standing in for the irregular grids the paper's
  method targets (Section I and V).  Off-diagonal values are
  ``-(0.5 + u)``, u in [0, 1), and the diagonal is ``sum|off| + 1``, so the
  matrix is symmetric and strictly diagonally dominant (hence SPD).  Removal
  and value draws come from SplitMix64 (Steele, Lea, Flood, "Fast
  splittable pseudorandom number generators", OOPSLA 2014) evaluated on a
  counter built from the unordered edge {i, j}, so the pair (i, j) and
  (j, i) always agree.
* vectors: ``numpy.random.default_rng(seed).uniform(-1, 1, n)``.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "CSR",
    "stencil27",
    "stencil27_irregular",
    "uniform_vector",
    "batched_grids",
    "splitmix64",
]


class CSR:
    """A CSR matrix held as three numpy arrays (row_ptr int64, col int32, val float64)."""

    __slots__ = ("n_rows", "n_cols", "row_ptr", "col", "val", "grid")

    def __init__(self, n_rows, n_cols, row_ptr, col, val, grid=None):
        self.n_rows = int(n_rows)
        self.n_cols = int(n_cols)
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        self.grid = grid

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1]) if self.row_ptr.size else 0

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def __repr__(self):
        return f"CSR({self.n_rows}x{self.n_cols}, nnz={self.nnz}, grid={self.grid})"


def _stencil_offsets():
    """The 27 (dz, dy, dx) triples in lexicographic order (= ascending column)."""
    out = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                out.append((dz, dy, dx))
    return out


def _stencil_structure(nx, ny, nz):
    """Return (row_ptr, cols as (n,27) with -1 for absent, valid mask (n,27))."""
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64)
    ix = idx % nx
    iy = (idx // nx) % ny
    iz = idx // (nx * ny)
    del idx
    valid = np.empty((n, 27), dtype=bool)
    cols = np.empty((n, 27), dtype=np.int32)
    base = np.arange(n, dtype=np.int64)
    for k, (dz, dy, dx) in enumerate(_stencil_offsets()):
        m = np.ones(n, dtype=bool)
        if dx:
            m &= (ix + dx >= 0) & (ix + dx < nx)
        if dy:
            m &= (iy + dy >= 0) & (iy + dy < ny)
        if dz:
            m &= (iz + dz >= 0) & (iz + dz < nz)
        valid[:, k] = m
        cols[:, k] = np.where(m, base + dz * nx * ny + dy * nx + dx, -1)
    return valid, cols


def stencil27(nx: int, ny: int, nz: int) -> CSR:
    """HPCG 27-point matrix on an nx*ny*nz grid: diagonal 26.0, neighbours -1.0."""
    if min(nx, ny, nz) < 1:
        raise ValueError("grid dimensions must be >= 1")
    n = nx * ny * nz
    valid, cols = _stencil_structure(nx, ny, nz)
    counts = valid.sum(axis=1, dtype=np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = cols[valid]  # row-major boolean indexing keeps per-row ascending order
    del cols
    vals = np.full((n, 27), -1.0)
    vals[:, 13] = 26.0  # (0,0,0) is the 14th offset in lexicographic order
    val = vals[valid]
    return CSR(n, n, row_ptr, col, val, grid=(nx, ny, nz))



def stencil_hierarchy(nx: int, ny: int, nz: int, n_levels: int):
    """Grid hierarchy of HPCG's multigrid problem: level l is the 27-point
    matrix on the (nx, ny, nz) / 2^l grid, and f2c[l] (int32, one entry per row
    of level l + 1) holds, for the coarse point (ix, iy, iz), the fine row of
    the point (2 ix, 2 iy, 2 iz).  Each side must be divisible by
    2^(n_levels - 1).  Returns (list of CSR, list of n_levels - 1 arrays)."""
    if n_levels < 1:
        raise ValueError("n_levels must be >= 1")
    step = 1 << (n_levels - 1)
    if nx % step or ny % step or nz % step:
        raise ValueError("grid sides must be divisible by 2^(n_levels - 1)")
    mats, f2c = [], []
    g = (nx, ny, nz)
    for lev in range(n_levels):
        mats.append(stencil27(*g))
        if lev + 1 < n_levels:
            cx, cy, cz = g[0] // 2, g[1] // 2, g[2] // 2
            i = np.arange(cx * cy * cz, dtype=np.int64)
            ix, iy, iz = i % cx, (i // cx) % cy, i // (cx * cy)
            f2c.append((2 * ix + g[0] * (2 * iy + g[1] * 2 * iz)).astype(np.int32))
            g = (cx, cy, cz)
    return mats, f2c

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied to uint64 state values (vectorised)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _edge_uniform(seed: int, lo: np.ndarray, hi: np.ndarray, n: int, stream: int) -> np.ndarray:
    """Uniform [0,1) from SplitMix64 at counter 2*(lo*n+hi)+stream+1 on the seeded stream."""
    c = lo.astype(np.uint64) * np.uint64(n) + hi.astype(np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed) * _GAMMA + (c * np.uint64(2) + np.uint64(stream + 1)) * _GAMMA
    bits = splitmix64(state) >> np.uint64(11)
    return bits.astype(np.float64) * (1.0 / 9007199254740992.0)


def stencil27_irregular(nx: int, ny: int, nz: int, seed: int = 0, p_remove: float = 0.05) -> CSR:
    """Irregularised 27-point matrix (symmetric, strictly diagonally dominant)."""
    n = nx * ny * nz
    valid, cols = _stencil_structure(nx, ny, nz)
    rows = np.broadcast_to(np.arange(n, dtype=np.int64)[:, None], (n, 27))
    offdiag = valid.copy()
    offdiag[:, 13] = False
    r = rows[offdiag]
    c = cols[offdiag].astype(np.int64)
    lo = np.minimum(r, c)
    hi = np.maximum(r, c)
    keep = _edge_uniform(seed, lo, hi, n, 0) >= p_remove
    offval = -(0.5 + _edge_uniform(seed, lo, hi, n, 1))
    del lo, hi
    keep_full = np.zeros((n, 27), dtype=bool)
    keep_full[offdiag] = keep
    keep_full[:, 13] = True
    vals = np.zeros((n, 27))
    vals[offdiag] = np.where(keep, offval, 0.0)
    # diagonal = sum of |off| in ascending column order, + 1
    diag = np.zeros(n)
    for k in range(27):
        if k != 13:
            diag += np.abs(vals[:, k])
    vals[:, 13] = diag + 1.0
    counts = keep_full.sum(axis=1, dtype=np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSR(n, n, row_ptr, cols[keep_full], vals[keep_full], grid=(nx, ny, nz))


def uniform_vector(n: int, seed: int = 0, dtype=np.float64) -> np.ndarray:
    """x ~ U[-1, 1] from ``numpy.random.default_rng(seed)``."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n).astype(dtype)


def batched_grids(n_sys: int = 64, lo: int = 16, hi: int = 96, seed: int = 0) -> list:
    """Grid dimensions for the batched workload: each axis uniform in [lo, hi]."""
    dims = np.random.default_rng(seed).integers(lo, hi + 1, size=(n_sys, 3))
    return [tuple(int(v) for v in d) for d in dims]
