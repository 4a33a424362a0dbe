"""Pins of the reference codec (the paper's Section V compression schemes).

* Fig. 1's worked example (V, S, T) from a golden fixture;
* the paper's bytes per 27-entry row (324 / 116 / 12, and about 4 once the
  values are registered in the table too);
* with the values registered (DITV), the signature count equals a brute-force
  count of distinct (displacements, codes) row sequences, IDs follow first
  occurrence, and the stencil gains no patterns (its T_i follows from the
  displacement pattern);
* the pattern count of the 27-point stencil, prod(min(n_a, 3)), and the rows
  per pattern, prod({1, n_a - 2, 1});
* lossless round trip, bit for bit, on random CSR matrices with special values;
* the paper's decode walk (sample code: value runs up to T, then j = i + d)
  reproduces the plain CSR product exactly on integer data.
"""
import itertools
import json
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from oracle import codec
from synthetic import CSR, stencil27, stencil27_irregular, uniform_vector

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def same_csr(A, B):
    return (A.n_rows == B.n_rows and A.n_cols == B.n_cols
            and np.array_equal(A.row_ptr, B.row_ptr) and np.array_equal(A.col, B.col)
            and np.array_equal(np.asarray(A.val).view(np.uint64), np.asarray(B.val).view(np.uint64)))


def test_fig1_worked_example():
    g = load("fig1_compression_example.json")
    cols = g["row_columns"]
    A = CSR(1, max(cols) + 1, [0, len(cols)], cols, g["row_values"])
    can = codec.canonicalize(A)
    assert can.V.tolist() == g["value_table"]
    assert can.S.tolist() == g["sorted_column_list"]
    assert (can.T[0] - 1).tolist() == g["terminal_indices_as_printed"]
    enc = codec.encode_dt(A)
    assert same_csr(codec.decode(enc), A)


def test_section5_row_bytes():
    g = load("section5_row_bytes.json")
    b = codec.paper_row_bytes(g["row_len"], g["value_table_size"])
    assert (b["ELL"], b["DT"], b["DIT"], b["DITV"]) == (g["ELL"], g["DT"], g["DIT"], g["DITV"])


def test_value_table_of_stencil_is_minus_one_and_26():
    A = stencil27(16, 16, 16)
    assert codec.value_table(A.val, A.n_rows).tolist() == [-1.0, 26.0]


@pytest.mark.parametrize("grid", [(16, 16, 16), (2, 5, 7), (1, 3, 4), (5, 4, 3), (3, 3, 3)])
def test_stencil_pattern_count(grid):
    A = stencil27(*grid)
    enc = codec.encode_dit(A, min_pattern_rows=1)
    assert enc.P == int(np.prod([min(m, 3) for m in grid]))
    assert enc.esc_rows.size == 0
    per_axis = [[1, m - 2, 1] if m >= 3 else [1] * m for m in grid]
    expect = sorted(int(np.prod(c)) for c in itertools.product(*per_axis))
    assert sorted(enc.pat_rows.tolist()) == expect
    # T of a stencil row: all -1 entries first, the diagonal 26 last
    lens = np.diff(A.row_ptr)
    assert np.array_equal(enc.T[:, 0], lens - 1) and np.array_equal(enc.T[:, 1], lens)


def test_stencil_default_rule_escapes_singleton_corners():
    A = stencil27(16, 16, 16)
    enc = codec.encode_dit(A)
    assert enc.P == 19 and enc.esc_rows.size == 8
    # pattern 0 is the first row's pattern (corner patterns are singletons and escape)
    assert enc.pat_first[0] == 1
    assert np.all(np.diff(enc.pat_first) > 0)


def test_pattern_ids_by_first_occurrence_and_cap():
    A = stencil27(10, 9, 8)
    full = codec.encode_dit(A, min_pattern_rows=1)
    assert np.all(np.diff(full.pat_first) > 0)
    capped = codec.encode_dit(A, min_pattern_rows=1, p_max=5)
    assert capped.P == 5
    # the five most frequent patterns survive, renumbered by first occurrence
    top = np.sort(full.pat_rows)[::-1][:5]
    assert sorted(capped.pat_rows.tolist(), reverse=True) == top.tolist()
    assert same_csr(codec.decode(capped), A)


@pytest.mark.parametrize("grid", [(16, 16, 16), (5, 4, 3), (1, 3, 4)])
def test_ditv_of_stencil_keeps_the_dit_patterns(grid):
    """A stencil row's T_i is fixed by its displacement pattern (the diagonal
    is the only 26), so registering the values adds no pattern: same IDs, and
    each pattern's T is (len - 1, len).  The row stream is the 1-byte ID."""
    A = stencil27(*grid)
    dit = codec.encode_dit(A, min_pattern_rows=1)
    ditv = codec.encode_dit(A, min_pattern_rows=1, fold_values=True)
    assert ditv.fmt == "DITV" and ditv.P == dit.P
    assert np.array_equal(ditv.ids, dit.ids) and np.array_equal(ditv.pat_off, dit.pat_off)
    plen = np.diff(ditv.pat_ptr)
    assert np.array_equal(ditv.pat_T, np.stack([plen - 1, plen], axis=1))
    assert codec.stream_bytes(ditv)["rows"] == A.n_rows
    assert same_csr(codec.decode(ditv), A)


def _signature_brute_force(A, V):
    """Per row, the tuple of (code, col - row) in (code, column) order -- the key
    a row registers when its values go into the table -- from the CSR, in plain
    Python; code K marks a raw value."""
    keys = []
    vb = [np.float64(v).view(np.uint64) for v in V]
    for i in range(A.n_rows):
        ent = []
        for k in range(int(A.row_ptr[i]), int(A.row_ptr[i + 1])):
            b = np.float64(A.val[k]).view(np.uint64)
            code = vb.index(b) if b in vb else len(V)
            ent.append((code, int(A.col[k]) - i))
        keys.append(tuple(sorted(ent)))
    return keys


def _scattered(p_v1):
    A = stencil27(6, 5, 4)
    rng = np.random.default_rng(17)
    A.val[:] = np.where(rng.random(A.nnz) < p_v1, 3.5, -1.0)
    return A


def _split_moves():
    """3-point rows whose values ascend with the column, so the (code, column)
    order is the column order for every row, but the split alternates:
    (-1, -1, 3.5) on even rows, (-1, 3.5, 3.5) on odd rows."""
    n = 12
    cols, vals, rp = [], [], [0]
    for i in range(n):
        c = [j for j in (i - 1, i, i + 1) if 0 <= j < n]
        v = [-1.0, -1.0, 3.5] if i % 2 == 0 else [-1.0, 3.5, 3.5]
        cols += c
        vals += v[3 - len(c):] if i == 0 else v[:len(c)]
        rp.append(len(cols))
    return CSR(n, n, np.array(rp), np.array(cols, dtype=np.int32), np.array(vals))


@pytest.mark.parametrize("make", [lambda: _scattered(0.0), lambda: _scattered(0.3), lambda: _scattered(0.5),
                                  _split_moves])
def test_ditv_signatures_brute_force(make):
    """Values from {-1, 3.5}: scattered per entry on a 27-point structure, or
    ascending along 3-point rows with a split that alternates between rows.
    The DITV pattern count is the number of distinct brute-force signatures,
    rows with equal signatures share an ID, IDs follow first occurrence,
    DIT's count is that of the displacement sequences (in (code, column)
    order) alone, and both decode to A."""
    A = make()
    rng = np.random.default_rng(18)
    ditv = codec.encode_dit(A, min_pattern_rows=1, fold_values=True)
    dit = codec.encode_dit(A, min_pattern_rows=1)
    keys = _signature_brute_force(A, ditv.V)
    first = {}
    for i, k in enumerate(keys):
        first.setdefault(k, i)
    assert ditv.P == len(first)
    order = sorted(first.values())
    expect = [order.index(first[k]) for k in keys]
    assert ditv.ids.tolist() == expect
    assert dit.P == len({tuple(d for _, d in k) for k in keys})  # DIT: the ordered displacements
    assert ditv.P >= dit.P
    if make is _split_moves:  # same displacement sequence, different T: DITV splits the pattern
        assert ditv.P > dit.P
    for enc in (dit, ditv):
        assert same_csr(codec.decode(enc), A)
    x = rng.integers(-50, 50, A.n_cols).astype(np.float64)
    assert np.array_equal(codec.walk_spmv(ditv, x), oracle.spmv(A, x))


def test_ditv_folded_table_decides_the_values():
    """Decoding a DITV encoding takes T from the pattern table: changing a
    pattern's registered T changes the decoded values, changing the per-row
    T (not part of the stream) does not."""
    A = stencil27(5, 5, 5)
    enc = codec.encode_dit(A, min_pattern_rows=1, fold_values=True)
    enc.T = np.zeros_like(enc.T)
    assert same_csr(codec.decode(enc), A)
    enc.pat_T = enc.pat_T.copy()
    enc.pat_T[0, 0] -= 1
    assert not same_csr(codec.decode(enc), A)


def test_paper_width_bytes_at_104():
    A = stencil27(104, 104, 104)
    enc = codec.encode_dit(A)
    sb = codec.stream_bytes(enc)
    n = A.n_rows
    assert sb["rows"] == 3 * n  # u8 ID + two u8 terminal indices
    assert codec.paper_row_bytes(27, 2)["DIT"] * n == 12 * n


# ---- lossless round trip ------------------------------------------------------------

SPECIAL = [0.0, -0.0, 1.0, -1.0, 26.0, np.inf, -np.inf, np.nan,
           np.frombuffer(np.uint64(0x7FF0000000000123).tobytes(), dtype=np.float64)[0],
           np.frombuffer(np.uint64(0xFFF8000000000042).tobytes(), dtype=np.float64)[0],
           5e-324, -1.7976931348623157e308]


@st.composite
def random_csr(draw):
    n_rows = draw(st.integers(0, 30))
    n_cols = draw(st.integers(1, 40))
    rows_cols = []
    for _ in range(n_rows):
        k = draw(st.integers(0, min(n_cols, 12)))
        rows_cols.append(sorted(draw(st.lists(st.integers(0, n_cols - 1), min_size=k, max_size=k,
                                              unique=True))))
    nnz = sum(len(c) for c in rows_cols)
    pool = draw(st.lists(st.sampled_from(SPECIAL) | st.floats(allow_nan=True, width=64),
                         min_size=1, max_size=6))
    vals = [draw(st.sampled_from(pool)) for _ in range(nnz)]
    rp = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum([len(c) for c in rows_cols], out=rp[1:])
    col = np.array([c for r in rows_cols for c in r], dtype=np.int32)
    val = np.array(vals, dtype=np.float64)
    return CSR(n_rows, n_cols, rp, col, val)


@settings(max_examples=150, deadline=None)
@given(random_csr(), st.integers(0, 4), st.integers(1, 3))
def test_roundtrip_random(A, k_max, min_rows):
    for enc in (codec.encode_dt(A, k_max=k_max),
                codec.encode_dit(A, k_max=k_max, min_pattern_rows=min_rows),
                codec.encode_dit(A, k_max=k_max, min_pattern_rows=min_rows, fold_values=True)):
        assert same_csr(codec.decode(enc), A)


def test_roundtrip_signed_zero_and_nan_payload_are_distinct_codes():
    nan_a = np.frombuffer(np.uint64(0x7FF8000000000001).tobytes(), dtype=np.float64)[0]
    nan_b = np.frombuffer(np.uint64(0x7FF8000000000002).tobytes(), dtype=np.float64)[0]
    vals = [0.0, -0.0, nan_a, nan_b] * 4
    rp = np.arange(0, 17, 4, dtype=np.int64)
    A = CSR(4, 4, rp, np.tile(np.arange(4), 4), vals)
    V = codec.value_table(A.val, A.n_rows)
    assert len(V) == 4
    keys = codec.total_order_key(V.view(np.uint64))
    assert np.all(np.diff(keys.astype(object)) > 0)
    assert V.view(np.uint64)[0] == np.float64(-0.0).view(np.uint64)  # -0 < +0 < NaNs
    for enc in (codec.encode_dt(A), codec.encode_dit(A)):
        assert same_csr(codec.decode(enc), A)


def test_roundtrip_irregular():
    A = stencil27_irregular(24, 20, 16, seed=0)
    enc = codec.encode_dit(A)
    assert enc.K == 0  # every value occurs at most twice: no value pays for a T byte
    assert same_csr(codec.decode(enc), A)
    assert 0 < enc.esc_rows.size < A.n_rows // 5


def test_long_rows_escape():
    n = 3
    rp = np.array([0, 300, 300, 301], dtype=np.int64)
    col = np.concatenate([np.arange(300), [2]]).astype(np.int32)
    A = CSR(n, 300, rp, col, np.ones(301))
    for enc in (codec.encode_dt(A), codec.encode_dit(A, min_pattern_rows=1)):
        assert 0 in enc.esc_rows.tolist()
        assert same_csr(codec.decode(enc), A)


# ---- decode walk (sample code in Section V) ------------------------------------------

@pytest.mark.parametrize("make", [lambda: stencil27(12, 11, 10),
                                  lambda: stencil27(16, 16, 16)])
def test_walk_spmv_exact_on_integer_data(make):
    A = make()
    x = np.random.default_rng(3).integers(-1000, 1000, A.n_cols).astype(np.float64)
    y = oracle.spmv(A, x)
    for enc in (codec.encode_dt(A), codec.encode_dit(A), codec.encode_dit(A, fold_values=True)):
        assert np.array_equal(codec.walk_spmv(enc, x), y)


def test_walk_spmv_inclusive_T_reading_fails():
    """Reading T as inclusive (as Fig. 1 prints it) drops one entry per value run."""
    A = stencil27(6, 6, 6)
    x = np.random.default_rng(4).integers(-9, 9, A.n_cols).astype(np.float64)
    enc = codec.encode_dit(A, min_pattern_rows=1)
    enc.T = enc.T - 1
    try:
        y = codec.walk_spmv(enc, x)
    except IndexError:  # the dropped entries fall into the (empty) raw stream
        return
    assert not np.array_equal(y, oracle.spmv(A, x))


def test_walk_spmv_irregular_close():
    A = stencil27_irregular(10, 9, 8, seed=5)
    x = uniform_vector(A.n_cols, seed=1)
    y = oracle.spmv(A, x)
    enc = codec.encode_dit(A)
    yw = codec.walk_spmv(enc, x)
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
    scale = np.bincount(rows, weights=np.abs(A.val) * np.abs(x[A.col]), minlength=A.n_rows)
    assert np.all(np.abs(yw - y) <= 1e-14 * scale)
