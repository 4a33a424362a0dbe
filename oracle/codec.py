"""Reference codec for the paper's compression schemes -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
use this module.  It shares no code with the GPU library.

It follows the steps of Section V in the paper's order:

1. Scan the whole matrix, list the unique element values and sort them in
   ascending order: the value table V (``value_table``).
2. Sort the non-zeros of every row by value; the column indices in that order
   are the sorted column list S_i (``canonicalize``).
3. For every v in V record where its run ends in S_i: the terminal indices
   T_i (``canonicalize``).  The "Data Table" scheme (DT) stores V, S, T.
4. Replace every column index by its displacement from the diagonal,
   d = col - row (``encode_dit``).
5. Register each row's displacement sequence in a pattern table; each row then
   stores only the pattern's type ID plus T_i.  This is the "Data+Index
   Table" scheme (DIT).  Decoding (Section V, Listing 1): the column of a
   row's k-th entry is the row index plus the k-th displacement of its
   pattern, and its value is the table value whose run in T_i covers k.
6. The further step the paper proposes at the end of the section: register
   the element values in the table as well, so that a row stores nothing but
   its ID (``encode_dit(..., fold_values=True)``, format "DITV").  Here the
   registered key is the displacement sequence together with T_i (which, with
   V fixed, determines the value of every coded entry); raw values stay per
   row as in DIT.

Readings of points the paper leaves open (each is listed in the design notes):

* T stores *exclusive* run ends (prefix counts).  The decoding loop of
  Listing 1 bounds each run with a strict comparison, which needs exclusive
  ends; Fig. 1 prints the inclusive last position, i.e. T - 1.
* Equal values keep ascending column order (a stable sort of a column-sorted
  row), which reproduces Fig. 1's S = 45 49 51 65 50.
* Values are compared by bit pattern and ordered by IEEE-754 totalOrder, so
  -0.0 and +0.0 are distinct and NaN payloads survive.
* The table is a dictionary of capacity ``k_max``: a value enters it when it
  pays for its T byte per row, i.e. 8 * count > n_rows, and only the
  ``k_max`` most frequent such values are kept (ties: totalOrder).  All other
  entries are "raw": ordered after the coded ones, by column, and stored as
  FP64 values per row.
* A pattern is the ordered displacement sequence (length included); with the
  values registered too it is that sequence plus T_i.  Pattern IDs are
  assigned by first occurrence (lowest row).  Rows whose pattern is
  used by fewer than ``min_pattern_rows`` rows, falls outside the ``p_max``
  most frequent patterns (ties: first occurrence), or whose length exceeds
  255 (T is one byte) are escape rows, kept as plain CSR.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

MAX_PATTERN_LEN = 255
SIGN = np.uint64(1) << np.uint64(63)


def total_order_key(bits) -> np.ndarray:
    """Map FP64 bit patterns to uint64 keys whose unsigned order is IEEE totalOrder."""
    bits = np.asarray(bits, dtype=np.uint64)
    neg = (bits & SIGN) != 0
    return np.where(neg, ~bits, bits | SIGN)


def _bits(val) -> np.ndarray:
    return np.ascontiguousarray(val, dtype=np.float64).view(np.uint64)


def value_table(val, n_rows: int, k_max: int = 15) -> np.ndarray:
    """Step 1: unique values -> dictionary V (ascending totalOrder), as float64."""
    bits = _bits(val)
    if bits.size == 0 or k_max <= 0:
        return np.zeros(0, dtype=np.float64)
    uniq, counts = np.unique(bits, return_counts=True)
    keep = 8 * counts.astype(np.int64) > int(n_rows)
    uniq, counts = uniq[keep], counts[keep].astype(np.int64)
    keys = total_order_key(uniq)
    order = np.lexsort((keys, -counts))[:k_max]  # most frequent first, ties by totalOrder
    sel = uniq[order]
    sel = sel[np.argsort(total_order_key(sel), kind="stable")]
    return sel.view(np.float64).copy()


def codes_of(val, V) -> np.ndarray:
    """Dictionary code of every entry: index into V, or K (= len(V)) for raw entries."""
    K = len(V)
    keys = total_order_key(_bits(val))
    if K == 0:
        return np.zeros(keys.shape, dtype=np.int64)
    vkeys = total_order_key(_bits(V))
    pos = np.searchsorted(vkeys, keys)
    hit = (pos < K) & (vkeys[np.minimum(pos, K - 1)] == keys)
    return np.where(hit, pos, K).astype(np.int64)


@dataclass
class Canonical:
    """Rows sorted by (code, column): S, per-row T (exclusive ends), raw values."""

    n_rows: int
    n_cols: int
    row_ptr: np.ndarray  # int64 [n+1], same as the input CSR
    V: np.ndarray  # float64 [K]
    S: np.ndarray  # int32 [nnz], columns in canonical order
    code: np.ndarray  # int64 [nnz], code of each canonical entry (K = raw)
    val: np.ndarray  # float64 [nnz], values in canonical order
    T: np.ndarray  # int64 [n, K], exclusive end of each code's run
    n_raw: np.ndarray  # int64 [n], raw entries per row (they follow T[:, K-1])

    @property
    def K(self) -> int:
        return len(self.V)


def _row_of(row_ptr: np.ndarray) -> np.ndarray:
    n = row_ptr.size - 1
    return np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))


def canonicalize(A, k_max: int = 15, V=None) -> Canonical:
    """Steps 1-3: V, then S_i (sorted by value, ties by column) and T_i per row."""
    n = A.n_rows
    rp = np.asarray(A.row_ptr, dtype=np.int64)
    if V is None:
        V = value_table(A.val, n, k_max)
    K = len(V)
    code = codes_of(A.val, V)
    row_of = _row_of(rp)
    # stable sort on (row, code); the input is column-ascending inside each row
    perm = np.argsort(row_of * (K + 1) + code, kind="stable")
    S = np.asarray(A.col, dtype=np.int32)[perm]
    code_c = code[perm]
    val_c = np.asarray(A.val, dtype=np.float64)[perm]
    cnt = np.bincount(row_of * (K + 1) + code, minlength=n * (K + 1)).reshape(n, K + 1)
    T = np.cumsum(cnt, axis=1)[:, :K].astype(np.int64)
    return Canonical(n, A.n_cols, rp.copy(), np.asarray(V, dtype=np.float64), S, code_c,
                     val_c, T, cnt[:, K].astype(np.int64))


@dataclass
class Encoding:
    """Logical content of a DT or DIT encoding (layout-independent)."""

    fmt: str  # "DT", "DIT" or "DITV" (DIT with the values registered in the table)
    n_rows: int
    n_cols: int
    V: np.ndarray  # float64 [K]
    T: np.ndarray  # int64 [n, K]; 0 on escape rows
    raw_ptr: np.ndarray  # int64 [n+1]; raw values of row i: raw[raw_ptr[i]:raw_ptr[i+1]]
    raw: np.ndarray  # float64, canonical order (ascending column) per row
    esc_rows: np.ndarray  # int64 [n_esc], ascending
    esc_ptr: np.ndarray  # int64 [n_esc+1]
    esc_col: np.ndarray  # int32
    esc_val: np.ndarray  # float64
    # DT only: sorted column list per non-escape row (CSR-shaped over all rows)
    S_ptr: np.ndarray = field(default=None)
    S: np.ndarray = field(default=None)
    # DIT only
    ids: np.ndarray = field(default=None)  # int64 [n], -1 = escape
    pat_ptr: np.ndarray = field(default=None)  # int64 [P+1]
    pat_off: np.ndarray = field(default=None)  # int64, displacements in canonical order
    pat_rows: np.ndarray = field(default=None)  # int64 [P], rows using each pattern
    pat_first: np.ndarray = field(default=None)  # int64 [P], first row using it
    # DITV only: T of each pattern (a row's T is its pattern's; the row stores no T)
    pat_T: np.ndarray = field(default=None)  # int64 [P, K]

    @property
    def K(self) -> int:
        return len(self.V)

    @property
    def P(self) -> int:
        return 0 if self.pat_ptr is None else self.pat_ptr.size - 1


def _escape_csr(A, esc_mask):
    rp = np.asarray(A.row_ptr, dtype=np.int64)
    esc_rows = np.flatnonzero(esc_mask).astype(np.int64)
    lens = rp[esc_rows + 1] - rp[esc_rows]
    esc_ptr = np.zeros(esc_rows.size + 1, dtype=np.int64)
    np.cumsum(lens, out=esc_ptr[1:])
    sel = np.repeat(esc_mask, np.diff(rp))
    return esc_rows, esc_ptr, np.asarray(A.col, np.int32)[sel].copy(), np.asarray(A.val)[sel].copy()


def _raw_stream(can: Canonical, keep_rows):
    n_raw = np.where(keep_rows, can.n_raw, 0)
    raw_ptr = np.zeros(can.n_rows + 1, dtype=np.int64)
    np.cumsum(n_raw, out=raw_ptr[1:])
    row_of = _row_of(can.row_ptr)
    sel = (can.code == can.K) & keep_rows[row_of]
    return raw_ptr, can.val[sel].copy()


def encode_dt(A, k_max: int = 15) -> Encoding:
    """The "Data Table" scheme: V, S_i, T_i per row (escapes: rows longer than 255)."""
    can = canonicalize(A, k_max)
    lens = np.diff(can.row_ptr)
    keep = lens <= MAX_PATTERN_LEN
    T = np.where(keep[:, None], can.T, 0)
    raw_ptr, raw = _raw_stream(can, keep)
    row_of = _row_of(can.row_ptr)
    sel = keep[row_of]
    S_ptr = np.zeros(can.n_rows + 1, dtype=np.int64)
    np.cumsum(np.where(keep, lens, 0), out=S_ptr[1:])
    er, ep, ec, ev = _escape_csr(A, ~keep)
    return Encoding("DT", can.n_rows, can.n_cols, can.V, T, raw_ptr, raw, er, ep, ec, ev,
                    S_ptr=S_ptr, S=can.S[sel].copy())


def encode_dit(A, k_max: int = 15, p_max: int = 65535, min_pattern_rows: int = 2,
               fold_values: bool = False) -> Encoding:
    """The "Data+Index Table" scheme: V, per-row pattern ID and T_i, pattern table.

    With ``fold_values`` the key registered per row is (displacements, T_i) and
    the row keeps only the ID (format "DITV"); ``T`` of the result is then the
    pattern's T repeated per row, for decoding, and is not part of the stream.
    """
    can = canonicalize(A, k_max)
    n = can.n_rows
    K = can.K
    rp = can.row_ptr
    lens = np.diff(rp)
    row_of = _row_of(rp)
    disp = can.S.astype(np.int64) - row_of  # step 4: displacement from the diagonal
    short = lens <= MAX_PATTERN_LEN
    short_rows = np.flatnonzero(short)
    W = int(lens[short].max()) if short_rows.size else 0
    # step 5: one row of M per row = (length, [T_i,] displacements..., 0 padding)
    H = 1 + (K if fold_values else 0)
    M = np.zeros((short_rows.size, W + H), dtype=np.int64)
    M[:, 0] = lens[short_rows]
    if fold_values and K:
        M[:, 1:H] = can.T[short_rows]
    if W > 0:
        ent = short[row_of]
        pos = np.arange(rp[-1], dtype=np.int64) - rp[row_of]
        slot = np.full(n, -1, dtype=np.int64)
        slot[short_rows] = np.arange(short_rows.size)
        M[slot[row_of[ent]], H + pos[ent]] = disp[ent]
    if short_rows.size:
        uniq, first, inv, cnt = np.unique(M, axis=0, return_index=True, return_inverse=True,
                                          return_counts=True)
        inv = inv.reshape(-1)
        first_row = short_rows[first]
    else:
        uniq = np.zeros((0, W + H), dtype=np.int64)
        first_row = np.zeros(0, dtype=np.int64)
        inv = np.zeros(0, dtype=np.int64)
        cnt = np.zeros(0, dtype=np.int64)
    kept = np.flatnonzero(cnt >= min_pattern_rows)
    if kept.size > p_max:
        order = np.lexsort((first_row[kept], -cnt[kept]))[:p_max]
        kept = kept[order]
    kept = kept[np.argsort(first_row[kept], kind="stable")]  # IDs by first occurrence
    pid = np.full(uniq.shape[0], -1, dtype=np.int64)
    pid[kept] = np.arange(kept.size)
    ids = np.full(n, -1, dtype=np.int64)
    ids[short_rows] = pid[inv]
    esc = ids < 0
    plen = uniq[kept, 0]
    pat_ptr = np.zeros(kept.size + 1, dtype=np.int64)
    np.cumsum(plen, out=pat_ptr[1:])
    pat_off = np.concatenate([uniq[u, H:H + uniq[u, 0]] for u in kept]) if kept.size else \
        np.zeros(0, dtype=np.int64)
    T = np.where(esc[:, None], 0, can.T)
    raw_ptr, raw = _raw_stream(can, ~esc)
    er, ep, ec, ev = _escape_csr(A, esc)
    pat_T = uniq[kept, 1:H].astype(np.int64) if fold_values else None
    return Encoding("DITV" if fold_values else "DIT", n, can.n_cols, can.V, T, raw_ptr, raw, er, ep, ec, ev,
                    ids=ids, pat_ptr=pat_ptr, pat_off=pat_off.astype(np.int64),
                    pat_rows=cnt[kept].astype(np.int64), pat_first=first_row[kept].astype(np.int64),
                    pat_T=pat_T)


def _entries(enc: Encoding):
    """(row, col, val) of every stored entry of an encoding, in canonical order per row."""
    n, K = enc.n_rows, enc.K
    if enc.fmt == "DT":
        lens = np.diff(enc.S_ptr)
    else:
        plen = np.diff(enc.pat_ptr)
        lens = np.where(enc.ids >= 0, plen[np.maximum(enc.ids, 0)] if plen.size else 0, 0)
    rows = np.repeat(np.arange(n, dtype=np.int64), lens)
    start = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=start[1:])
    k = np.arange(start[-1], dtype=np.int64) - start[rows]
    if enc.fmt == "DT":
        cols = enc.S.astype(np.int64)
    else:
        cols = rows + enc.pat_off[enc.pat_ptr[enc.ids[rows]] + k]
    # DITV: T_i comes from the row's pattern, not from a per-row stream
    Tr = enc.pat_T[enc.ids[rows]] if enc.fmt == "DITV" else enc.T[rows]  # [m, K]
    code = (k[:, None] >= Tr).sum(axis=1) if K else np.zeros(rows.size, dtype=np.int64)
    vals = np.empty(rows.size, dtype=np.float64)
    coded = code < K
    vals[coded] = enc.V[code[coded]]
    raw_k = k - (Tr[:, K - 1] if K else 0)
    vals[~coded] = enc.raw[enc.raw_ptr[rows[~coded]] + raw_k[~coded]]
    er = np.repeat(enc.esc_rows, np.diff(enc.esc_ptr))
    return (np.concatenate([rows, er]), np.concatenate([cols, enc.esc_col.astype(np.int64)]),
            np.concatenate([vals, enc.esc_val]))


def decode(enc: Encoding):
    """Rebuild the CSR matrix (columns ascending per row) from a DT/DIT encoding."""
    from synthetic import CSR  # the container type only; no arithmetic

    rows, cols, vals = _entries(enc)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rp = np.zeros(enc.n_rows + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=enc.n_rows), out=rp[1:])
    return CSR(enc.n_rows, enc.n_cols, rp, cols.astype(np.int32), vals)


def walk_spmv(enc: Encoding, x) -> np.ndarray:
    """y = A x evaluated from the encoding itself (not from the CSR input).

    Every stored entry is decoded by ``_entries`` -- its column from the row's
    pattern (DIT, DITV) or S_i (DT), its value from V through T_i or from the
    raw stream, escape rows from their CSR -- and y_i is then the plain sum of
    value * x[column] over row i's entries, added in their stored order.
    """
    x = np.asarray(x, dtype=np.float64)
    rows, cols, vals = _entries(enc)
    y = np.zeros(enc.n_rows, dtype=np.float64)
    np.add.at(y, rows, vals * x[cols])  # unbuffered: in index order, one entry at a time
    return y


# ---- byte accounting -------------------------------------------------------------------

def paper_row_bytes(row_len: int, K: int) -> dict:
    """Bytes per row at the paper's widths (4-byte indices, 8-byte values).

    ELL: (4 + 8) per element; DT: (len + K) * 4 (S_i and T_i); DIT: one 4-byte
    type ID plus T_i, (1 + K) * 4; DITV (values registered in the table too):
    the 4-byte ID alone (Section V).
    """
    return {"ELL": 12 * row_len, "DT": (row_len + K) * 4, "DIT": 4 * (1 + K), "DITV": 4}


def id_width(P: int) -> int:
    """Smallest unsigned width (bytes) holding IDs 0..P-1 plus one escape marker."""
    if P <= 255:
        return 1
    if P <= 65535:
        return 2
    return 4


def stream_bytes(enc: Encoding) -> dict:
    """Logical per-matrix byte counts of an encoding at the actual (narrow) widths."""
    n, K = enc.n_rows, enc.K
    esc = 12 * int(enc.esc_col.size) + 16 * int(enc.esc_rows.size)
    raw = 8 * int(enc.raw.size)
    table = 8 * K
    if enc.fmt == "DT":
        rows = 4 * int(enc.S.size) + K * n
    elif enc.fmt == "DIT":
        rows = id_width(enc.P) * n + K * n
        table += 4 * int(enc.pat_off.size) + 4 * enc.P
    else:  # DITV: the row holds its ID only; T_i lives in the table
        rows = id_width(enc.P) * n
        table += 4 * int(enc.pat_off.size) + 4 * enc.P + K * enc.P
    return {"rows": rows, "raw": raw, "escape": esc, "table": table,
            "total": rows + raw + esc + table}
