"""GPU parity of compression and SpMV against the CPU oracle (called through the C ABI).

* compression is lossless: decompress(compress(A)) == A bit for bit;
* the encoded arrays equal the reference codec's (deterministic IDs, exact V/T);
* FP64 SpMV within 1e-14 of the oracle, per row relative to sum |a_ij||x_j|;
* FP32 SpMV within (len + 2) * 2^-24 of the same normaliser;
* block SpMV equals the oracle's per-column products.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import codec
from synthetic import CSR, stencil27, stencil27_irregular, uniform_vector

from gpu_util import compress, lib, max_rel_err, row_scale, same_bits, torch_mod

pytestmark = pytest.mark.gpu

FORMATS = ["ELL", "DT", "DIT", "DITV"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_spmv(M, x, dtype="f64"):
    torch = torch_mod()
    t = torch.from_numpy(x).cuda()
    if dtype == "f32":
        t = t.float()
    y = M.spmv(t)
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


def roundtrip_ok(M, A):
    rp, col, val = M.decompress()
    return (np.array_equal(rp.cpu().numpy(), A.row_ptr) and np.array_equal(col.cpu().numpy(), A.col)
            and same_bits(val.cpu().numpy(), A.val))


def _scattered_two_values(grid=(16, 13, 11), p_v1=0.3, seed=11):
    """27-point structure, values drawn per entry from {-1, 3.5} (seeded)."""
    A = stencil27(*grid)
    rng = np.random.default_rng(seed)
    A.val[:] = np.where(rng.random(A.nnz) < p_v1, 3.5, -1.0)
    return A


def _split_alternates(n=200):
    """3-point rows whose values ascend with the column, split alternating
    between rows: (-1, -1, 3.5) and (-1, 3.5, 3.5) -- one DIT pattern, two DITV ones."""
    cols, vals, rp = [], [], [0]
    for i in range(n):
        c = [j for j in (i - 1, i, i + 1) if 0 <= j < n]
        v = [-1.0, -1.0, 3.5] if i % 2 == 0 else [-1.0, 3.5, 3.5]
        cols += c
        vals += v[3 - len(c):] if i == 0 else v[:len(c)]
        rp.append(len(cols))
    return CSR(n, n, np.array(rp), np.array(cols, dtype=np.int32), np.array(vals))


@pytest.mark.parametrize("fmt", FORMATS)
def test_stencil16_parity_and_roundtrip(fmt):
    say("case: stencil 16^3", fmt)
    A = stencil27(16, 16, 16)
    x = uniform_vector(A.n_cols, seed=0)
    M = compress(A, fmt=fmt)
    y = gpu_spmv(M, x)
    assert max_rel_err(A, x, y, oracle.spmv(A, x)) <= 1e-14
    assert roundtrip_ok(M, A)


@pytest.mark.parametrize("fmt", FORMATS)
def test_stencil104_full_size_parity(fmt):
    say("case: stencil 104^3", fmt)
    A = stencil27(104, 104, 104)
    x = uniform_vector(A.n_cols, seed=0)
    M = compress(A, fmt=fmt)
    y = gpu_spmv(M, x)
    assert max_rel_err(A, x, y, oracle.spmv(A, x)) <= 1e-14
    inf = M.info()
    if fmt in ("DIT", "DITV"):
        assert inf["K"] == 2 and inf["P"] == 19 and inf["n_escape_rows"] == 8
        assert inf["id_bytes"] == 1 and inf["lds_windows"] == 3
    if fmt == "DITV":  # the row stream is the 1-byte ID alone
        dit = compress(A, fmt="DIT").info()
        assert inf["fmt_name"] == "DITV" and M.array("T").numel() == 0
        assert dit["bytes_stream"] - inf["bytes_stream"] == 2 * ((A.n_rows + 63) // 64 * 64) - 2 * inf["P"]
    # closed form: A*1 = 26 - #neighbours, exact in any summation order
    y1 = gpu_spmv(M, np.ones(A.n_cols))
    assert np.array_equal(y1, oracle.spmv(A, np.ones(A.n_cols)))
    assert roundtrip_ok(M, A)


@pytest.mark.parametrize("rows,lds", [(256, 1), (512, 1), (768, 1), (1024, 1), (2048, 1), (4096, 1), (1024, 0),
                                      (256, 2), (512, 2), (1024, 2)])
def test_dit_kernel_configs_agree(rows, lds):
    say("case: DIT config", rows, lds)
    A = stencil27(40, 37, 23)
    x = uniform_vector(A.n_cols, seed=3)
    M = compress(A, fmt="DIT")
    M.set_config(rows, lds)
    y = gpu_spmv(M, x)
    assert max_rel_err(A, x, y, oracle.spmv(A, x)) <= 1e-14


@pytest.mark.parametrize("grid,rows", [((104, 104, 104), 256), ((104, 104, 104), 512), ((104, 104, 104), 1024),
                                       ((61, 17, 33), 256), ((128, 128, 128), 512)])
def test_plane_marching_equals_register_kernel(grid, rows):
    """The plane-marching kernel computes every row with the register kernel's
    code, so y agrees bit for bit; also with x not 16-byte aligned (windows
    copied through registers) and in FP32.  61 x 17: planes of 1037 rows; the
    march steps by the spacing of the 4-aligned windows (1036 or 1040 rows),
    which partitions the rows just as well."""
    say("case: plane marching vs register", grid, rows)
    torch = torch_mod()
    A = stencil27(*grid)
    xh = uniform_vector(A.n_cols, seed=9)
    M = compress(A, fmt="DIT")
    marching = True
    buf = torch.zeros(A.n_cols + 1, dtype=torch.float64, device="cuda")
    buf[1:] = torch.from_numpy(xh).cuda()
    for x in (buf[1:].clone(), buf[1:]):
        M.set_config(rows, 1)
        y_reg = M.spmv(x).cpu().numpy()
        M.set_config(rows, 2)
        assert M.info()["kernel_name"] == ("k_dit_march" if marching else "k_dit_reg")
        y_m = M.spmv(x).cpu().numpy()
        assert same_bits(y_m, y_reg)
        assert max_rel_err(A, xh, y_m, oracle.spmv(A, xh)) <= 1e-14
        x32 = x.float()
        M.set_config(rows, 1)
        y32 = M.spmv(x32).cpu().numpy()
        M.set_config(rows, 2)
        assert same_bits(M.spmv(x32).cpu().numpy(), y32)


def test_plane_marching_raw_values_irregular():
    """Every value raw (K = 0): the marching kernel's raw path against the oracle."""
    say("case: plane marching, irregular 128^3")
    A = stencil27_irregular(128, 128, 128, seed=0)
    x = uniform_vector(A.n_cols, seed=4)
    M = compress(A, fmt="DIT")
    M.set_config(512, 1)
    y_reg = gpu_spmv(M, x)
    M.set_config(512, 2)
    assert M.info()["kernel_name"] == "k_dit_march"
    y_m = gpu_spmv(M, x)
    assert max_rel_err(A, x, y_m, oracle.spmv(A, x)) <= 1e-14
    assert same_bits(y_m, y_reg)


@pytest.mark.parametrize("fmt", FORMATS)
def test_irregular128_parity_and_roundtrip(fmt):
    say("case: irregular 128^3", fmt)
    A = stencil27_irregular(128, 128, 128, seed=0)
    x = uniform_vector(A.n_cols, seed=0)
    M = compress(A, fmt=fmt)
    y = gpu_spmv(M, x)
    assert max_rel_err(A, x, y, oracle.spmv(A, x)) <= 1e-14
    assert roundtrip_ok(M, A)
    if fmt in ("DIT", "DITV"):
        inf = M.info()
        assert inf["K"] == 0 and inf["id_bytes"] == 2
        assert inf["n_escape_rows"] < 0.02 * A.n_rows


@pytest.mark.parametrize("fmt", FORMATS)
def test_fp32_within_bound(fmt):
    say("case: fp32", fmt)
    for A in (stencil27(33, 20, 17), stencil27_irregular(24, 22, 20, seed=2)):
        x = uniform_vector(A.n_cols, seed=1).astype(np.float32)
        M = compress(A, fmt=fmt)
        y = gpu_spmv(M, x.astype(np.float64), dtype="f32")
        yref = oracle.spmv(A, x.astype(np.float64))
        lens = np.diff(A.row_ptr)
        s = row_scale(A, x.astype(np.float64))
        assert np.all(np.abs(y - yref) <= (lens + 2) * 2.0 ** -24 * s + 1e-300)


def _fp32_bound_ok(A, x32, y, yref, scale):
    """|y - yref| <= (len + 2) 2^-24 sum |a||x| per row: V is exact in FP32 and
    x is FP32, so every product is exact in FP64 and only the FP32 sums round."""
    lens = np.diff(A.row_ptr)
    return bool(np.all(np.abs(y - yref) <= (lens + 2) * 2.0 ** -24 * scale + 1e-300))


@pytest.mark.parametrize("grid", [(104, 104, 104), (192, 192, 192)])
def test_fp32_full_size_every_configuration(grid):
    """FP32 SpMV element by element against the oracle at the workloads' own
    sizes (104^3: the SpMV benchmark; 192^3: the inner SpMV of mixed-precision
    CG) in every FP32 kernel configuration the tuner can pick -- register
    kernel and plane marching at 256, 512 and 1024 rows per block, the direct
    gather -- and in the tuned one."""
    say("case: fp32 full size", grid)
    torch = torch_mod()
    A = stencil27(*grid)
    x32 = uniform_vector(A.n_cols, seed=5).astype(np.float32)
    x64 = x32.astype(np.float64)
    yref = oracle.spmv(A, x64)
    absA = CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, np.abs(A.val))
    scale = oracle.spmv(absA, np.abs(x64))
    M = compress(A, fmt="DIT")
    xt = torch.from_numpy(x32).cuda()
    for rows, lds in [(256, 1), (512, 1), (768, 1), (1024, 1), (256, 2), (512, 2), (1024, 2), (512, 0),
                      (None, None)]:
        if rows is None:
            M.tune(torch.float32)
        else:
            M.set_config(rows, lds)
        say("  config", rows, lds, M.info()["kernel_name_f32"])
        y = M.spmv(xt)
        torch.cuda.synchronize()
        assert _fp32_bound_ok(A, x32, y.double().cpu().numpy(), yref, scale), (rows, lds)


def test_fp32_table_value_beyond_float_range():
    """A table value finite in FP64 but above the FP32 range (1e39) becomes
    +inf in the FP32 copy of V.  FP32 SpMV must then give +-inf on the rows
    holding it (the sign of that row's x) and never NaN: a padded slot of a
    short row must not multiply inf by the zero window."""
    say("case: fp32 value beyond float range")
    torch = torch_mod()
    A = stencil27(40, 37, 23)
    A.val[A.val == 26.0] = 1e39
    x32 = uniform_vector(A.n_cols, seed=6).astype(np.float32)
    x32[x32 == 0] = 0.5
    M = compress(A, fmt="DIT")
    assert sorted(M.info()["V"][:2]) == [-1.0, 1e39]
    for rows, lds in [(512, 1), (512, 2), (512, 0)]:
        M.set_config(rows, lds)
        y = M.spmv(torch.from_numpy(x32).cuda())
        torch.cuda.synchronize()
        y = y.cpu().numpy()
        assert not np.isnan(y).any(), (rows, lds)
        assert np.array_equal(y, np.where(x32 > 0, np.inf, -np.inf).astype(np.float32)), (rows, lds)


@pytest.mark.parametrize("fmt", FORMATS)
@pytest.mark.parametrize("nrhs", [1, 3, 8, 16])
def test_block_spmv(fmt, nrhs):
    say("case: block", fmt, nrhs)
    torch = torch_mod()
    A = stencil27_irregular(20, 18, 15, seed=4) if fmt == "DT" else stencil27(21, 18, 15)
    X = np.stack([uniform_vector(A.n_cols, seed=10 + r) for r in range(nrhs)], axis=1)
    M = compress(A, fmt=fmt)
    Y = M.spmv_block(torch.from_numpy(X).cuda())
    torch.cuda.synchronize()
    Y = Y.cpu().numpy()
    Yref = oracle.spmv_block(A, X)
    for r in range(nrhs):
        assert max_rel_err(A, X[:, r], Y[:, r], Yref[:, r]) <= 1e-14


@pytest.mark.parametrize("fmt", FORMATS)
@pytest.mark.parametrize("nrhs,ld,off", [(8, 11, 0), (6, 8, 1), (2, 2, 0), (5, 5, 0), (4, 6, 0)])
def test_block_spmv_strided_and_unaligned(fmt, nrhs, ld, off):
    """Blocks with a leading dimension above nrhs (odd or even) and blocks that
    start one element into their buffer (not 16-byte aligned): the pair-wise
    lane loads are taken only when every row's pair is aligned, else single
    loads; irregular values (raw FP64) for DIT and DT, stencil for ELL."""
    say("case: block strided", fmt, nrhs, ld, off)
    torch = torch_mod()
    A = stencil27(21, 18, 15) if fmt == "ELL" else stencil27_irregular(20, 18, 15, seed=4)
    X = np.stack([uniform_vector(A.n_cols, seed=30 + r) for r in range(nrhs)], axis=1)
    M = compress(A, fmt=fmt)
    xb = torch.zeros(A.n_cols * ld + off, dtype=torch.float64, device="cuda")
    xv = xb[off:].view(A.n_cols, ld)[:, :nrhs]
    xv.copy_(torch.from_numpy(X).cuda())
    yb = torch.full((A.n_rows * ld + off,), 7.0, dtype=torch.float64, device="cuda")
    yv = yb[off:].view(A.n_rows, ld)[:, :nrhs]
    M.spmv_block(xv, yv)
    torch.cuda.synchronize()
    Y = yv.cpu().numpy()
    Yref = oracle.spmv_block(A, X)
    for r in range(nrhs):
        assert max_rel_err(A, X[:, r], Y[:, r], Yref[:, r]) <= 1e-14
    # columns past nrhs are untouched
    if ld > nrhs:
        assert np.all(yb[off:].view(A.n_rows, ld)[:, nrhs:].cpu().numpy() == 7.0)


@pytest.mark.parametrize("mode,grid,nrhs,ld", [(2, (104, 104, 104), 8, 8), (2, (33, 29, 17), 4, 10),
                                               (2, (33, 29, 17), 16, 16), (3, (104, 104, 104), 8, 8),
                                               (3, (33, 29, 17), 4, 4), (3, (33, 29, 17), 2, 2),
                                               (3, (33, 29, 17), 8, 10)])
def test_block_lds_kernels(mode, grid, nrhs, ld):
    """FP64 block SpMV through the LDS kernels (tuner candidates for DIT
    matrices): mode 2, windows of right-hand-side pairs; mode 3, whole rows one
    window at a time (unpadded blocks of 2, 4 or 8; a padded block falls back).
    104^3 at full size with 8 right-hand sides, every element checked against
    the oracle.  Escape rows (the 8 singleton corners) take their own launch."""
    say("case: block lds", mode, grid, nrhs, ld)
    torch = torch_mod()
    A = stencil27(*grid)
    X = np.stack([uniform_vector(A.n_cols, seed=60 + r) for r in range(nrhs)], axis=1)
    M = compress(A, fmt="DIT")
    assert M.info()["n_escape_rows"] == 8
    assert M.info()["block_split"] == 1  # every stencil row ends its canonical order with the diagonal
    M.set_block_mode(mode)
    xb = torch.zeros((A.n_cols, ld), dtype=torch.float64, device="cuda")
    xb[:, :nrhs] = torch.from_numpy(X).cuda()
    yb = torch.full((A.n_rows, ld), 5.0, dtype=torch.float64, device="cuda")
    M.spmv_block(xb[:, :nrhs], yb[:, :nrhs])
    torch.cuda.synchronize()
    Y = yb[:, :nrhs].cpu().numpy()
    Yref = oracle.spmv_block(A, X)
    for r in range(nrhs):
        assert max_rel_err(A, X[:, r], Y[:, r], Yref[:, r]) <= 1e-14
    if ld > nrhs:
        assert np.all(yb[:, nrhs:].cpu().numpy() == 5.0)


@pytest.mark.parametrize("make", [_scattered_two_values, _split_alternates,
                                  lambda: stencil27(40, 37, 23)])
def test_ditv_equals_dit_in_every_kernel(make):
    """DITV rows take T_i from their pattern (the register kernels from the
    pattern row's header word, the others from the pattern's T bytes); the
    entry order and the arithmetic are DIT's, so y is DIT's bit for bit in
    every single-vector configuration (register, plane-marching, LDS walk,
    direct gather; FP64 and FP32) and every block kernel, and within the bound
    of the oracle.  Rows that escape in either format (a pattern that DITV
    splits may fall under the two-row rule) are summed in CSR order there and
    are compared with the oracle only."""
    say("case: DITV vs DIT")
    torch = torch_mod()
    A = make()
    Md, Mv = compress(A, fmt="DIT"), compress(A, fmt="DITV")
    # (with the default escape rule a split pattern may fall under two rows and
    # escape, so DITV can keep fewer patterns than DIT)
    assert Mv.info()["fmt_name"] == "DITV" and Mv.info()["P"] == codec.encode_dit(A, fold_values=True).P
    both = np.ones(A.n_rows, dtype=bool)  # rows on a pattern in both formats
    for M in (Md, Mv):
        both[_np(M.array("ESC_ROWS"), np.int64)] = False
    x = uniform_vector(A.n_cols, seed=21)
    ref = oracle.spmv(A, x)
    for rows, lds in ((256, 1), (512, 1), (1024, 1), (2048, 1), (512, 0), (256, 2), (512, 2)):
        Md.set_config(rows, lds)
        Mv.set_config(rows, lds)
        assert Mv.info()["kernel_name"] == Md.info()["kernel_name"]
        yv = gpu_spmv(Mv, x)
        assert same_bits(yv[both], gpu_spmv(Md, x)[both])
        assert max_rel_err(A, x, yv, ref) <= 1e-14
        assert same_bits(gpu_spmv(Mv, x, "f32")[both], gpu_spmv(Md, x, "f32")[both])
    for mode in (3, 2, 1, 0):
        Md.set_block_mode(mode)
        Mv.set_block_mode(mode)
        for nrhs in (2, 8):
            X = torch.from_numpy(np.stack([uniform_vector(A.n_cols, seed=30 + r) for r in range(nrhs)], 1)).cuda()
            Yv = Mv.spmv_block(X).cpu().numpy()
            # the window-phased kernel sums per value run where every pattern's
            # rows share their split (always for DITV) and weights each entry
            # otherwise: the two forms add in different orders
            if mode != 3 or Mv.info()["block_split"] == Md.info()["block_split"]:
                assert same_bits(Yv[both], Md.spmv_block(X).cpu().numpy()[both])
            Yref = oracle.spmv_block(A, X.cpu().numpy())
            for r in range(nrhs):
                assert max_rel_err(A, X[:, r].cpu().numpy(), Yv[:, r], Yref[:, r]) <= 1e-14


@pytest.mark.parametrize("mode", [3, 2, 1, 0])
def test_block_spmv_scattered_two_value_dictionary(mode):
    """A 27-point structure whose values are drawn per entry from {-1, 3.5}
    (seeded): K = 2 with the V[1] entries anywhere in a row, so within one
    pattern the split point T changes from row to row and the V[1] entries of
    a window are not the same ones from row to row.  Every block kernel (and
    the single-vector kernels) must weight each product by its own entry."""
    say("case: block scattered dictionary", mode)
    torch = torch_mod()
    A = stencil27(33, 29, 17)
    rng = np.random.default_rng(11)
    A.val[:] = np.where(rng.random(A.nnz) < 0.3, 3.5, -1.0)
    M = compress(A, fmt="DIT")
    assert M.info()["K"] == 2
    assert M.info()["block_split"] == 0  # rows of one pattern split differently: a weight per entry
    assert compress(A, fmt="DITV").info()["block_split"] == 1  # DITV: the split is the pattern's
    M.set_block_mode(mode)
    for nrhs in (2, 8):
        X = np.stack([uniform_vector(A.n_cols, seed=80 + r) for r in range(nrhs)], axis=1)
        Y = M.spmv_block(torch.from_numpy(X).cuda()).cpu().numpy()
        Yref = oracle.spmv_block(A, X)
        for r in range(nrhs):
            assert max_rel_err(A, X[:, r], Y[:, r], Yref[:, r]) <= 1e-14
    x = uniform_vector(A.n_cols, seed=90)
    assert max_rel_err(A, x, gpu_spmv(M, x), oracle.spmv(A, x)) <= 1e-14


def test_autotuner_single_and_block():
    """The autotuner's choices (single vector: rows per block / staging; block:
    lane group or one lane per row) keep every product within the bound."""
    say("case: autotuner")
    torch = torch_mod()
    A = stencil27(48, 40, 36)
    M = compress(A, fmt="DIT")
    x = uniform_vector(A.n_cols, seed=2)
    X = np.stack([uniform_vector(A.n_cols, seed=40 + r) for r in range(8)], axis=1)
    for dt in (torch.float64, torch.float32):
        t = M.tune(dt)
        assert t["rows_per_block"] in (256, 512, 1024, 2048, 4096) and t["lds"] in (0, 1, 2) and t["us"] > 0
    tb = M.tune(torch.float64, nrhs=8)
    assert tb["lds"] in (0, 1, 2, 3) and tb["us"] > 0
    assert max_rel_err(A, x, gpu_spmv(M, x), oracle.spmv(A, x)) <= 1e-14
    Y = M.spmv_block(torch.from_numpy(X).cuda()).cpu().numpy()
    Yref = oracle.spmv_block(A, X)
    for r in range(8):
        assert max_rel_err(A, X[:, r], Y[:, r], Yref[:, r]) <= 1e-14


# ---- encoded arrays equal the reference codec's -----------------------------------------

def _np(t, dtype):
    return t.cpu().numpy().view(dtype)


@pytest.mark.parametrize("fmt,make", [("DIT", lambda: stencil27(16, 16, 16)),
                                      ("DIT", lambda: stencil27_irregular(20, 17, 13, seed=1)),
                                      ("DIT", lambda: stencil27(5, 3, 4)),
                                      ("DITV", lambda: stencil27(16, 16, 16)),
                                      ("DITV", lambda: stencil27_irregular(20, 17, 13, seed=1)),
                                      ("DITV", lambda: _scattered_two_values((9, 8, 7), 0.02)),
                                      ("DITV", _split_alternates),
                                      ("DIT", "irregular128"), ("DITV", "irregular128")])
def test_dit_arrays_equal_reference_codec(fmt, make):
    """Every array of the GPU encoding equals the reference codec's: V, IDs, T
    (or the patterns' T for DITV), the pattern table, the escape CSR and the
    raw values of every row.  The full irregular 128^3 matrix (53 M entries,
    20,017 patterns, 17,599 escape rows) exercises candidate ranking, the
    two-row rule and the escape path at the workload's own size."""
    say("case: DIT arrays", fmt, make if isinstance(make, str) else "")
    A = stencil27_irregular(128, 128, 128, seed=0) if make == "irregular128" else make()
    enc = codec.encode_dit(A, fold_values=fmt == "DITV")
    M = compress(A, fmt=fmt)
    inf = M.info()
    n, n_pad, K, W = A.n_rows, ((A.n_rows + 63) // 64) * 64, enc.K, inf["width"]
    assert inf["K"] == K and inf["P"] == enc.P
    assert same_bits(np.array(inf["V"]), enc.V)
    idt = {1: np.uint8, 2: np.uint16, 4: np.uint32}[inf["id_bytes"]]
    ids = _np(M.array("IDS"), idt)[:n].astype(np.int64)
    ids[ids == np.iinfo(idt).max] = -1
    assert np.array_equal(ids, enc.ids)
    if K and fmt == "DIT":
        T = _np(M.array("T"), np.uint8).reshape(K, n_pad)[:, :n].T
        assert np.array_equal(T, enc.T)
    if fmt == "DITV":  # no per-row T; the patterns carry it
        assert M.array("T").numel() == 0
        if K and enc.P:
            pT = _np(M.array("PAT_T"), np.uint8)[:enc.P * K].reshape(enc.P, K).astype(np.int64)
            assert np.array_equal(pT, enc.pat_T)
        assert roundtrip_ok(M, A)
    pl = _np(M.array("PAT_LEN"), np.uint8).astype(np.int64)
    assert np.array_equal(pl, np.diff(enc.pat_ptr))
    po = _np(M.array("PAT_OFF"), np.int32).reshape(enc.P, W)
    used = np.arange(W)[None, :] < pl[:, None]  # row-major: the patterns one after another
    assert np.array_equal(po[used], enc.pat_off)
    assert np.array_equal(_np(M.array("ESC_ROWS"), np.int64), enc.esc_rows)
    if enc.esc_rows.size:
        assert np.array_equal(_np(M.array("ESC_PTR"), np.int64), enc.esc_ptr)
        assert np.array_equal(_np(M.array("ESC_COL"), np.int32)[:enc.esc_col.size], enc.esc_col)
        assert same_bits(_np(M.array("ESC_VAL"), np.float64)[:enc.esc_val.size], enc.esc_val)
    # raw values of every row: slices of 64 rows, column-major inside a slice
    if enc.raw.size:
        raw = _np(M.array("RAW"), np.float64)
        sl = _np(M.array("RAW_SLICE"), np.int64)
        k = np.diff(enc.raw_ptr)
        rows = np.repeat(np.arange(n, dtype=np.int64), k)
        j = np.arange(enc.raw.size, dtype=np.int64) - enc.raw_ptr[rows]
        assert same_bits(raw[sl[rows // 64] + rows % 64 + 64 * j], enc.raw)


@pytest.mark.parametrize("fmt", ["DIT", "DITV"])
def test_pattern_hash_collisions_are_resolved(fmt, monkeypatch):
    """With the first attempt's pattern hash narrowed to 4 bits (a test switch
    of the compressor), different displacement sequences collide; the
    compressor must detect it and hash again with a new seed, giving the very
    arrays of the reference codec and a bit-exact round trip."""
    say("case: pattern hash collisions", fmt)
    monkeypatch.setenv("SPMVC_TEST_WEAK_PATTERN_HASH", "1")
    for make in (lambda: stencil27(16, 16, 16), lambda: stencil27_irregular(20, 17, 13, seed=1)):
        test_dit_arrays_equal_reference_codec(fmt, make)
        A = make()
        M = compress(A, fmt=fmt)
        assert roundtrip_ok(M, A)
        x = uniform_vector(A.n_cols, seed=2)
        assert max_rel_err(A, x, gpu_spmv(M, x), oracle.spmv(A, x)) <= 1e-14


def test_dt_arrays_equal_reference_codec():
    say("case: DT arrays")
    A = stencil27(12, 10, 9)
    enc = codec.encode_dt(A)
    M = compress(A, fmt="DT")
    inf = M.info()
    n, n_pad, W = A.n_rows, ((A.n_rows + 63) // 64) * 64, inf["width"]
    S = _np(M.array("DT_S"), np.int32).reshape(W, n_pad)[:, :n].T
    for i in range(n):
        L = enc.S_ptr[i + 1] - enc.S_ptr[i]
        assert np.array_equal(S[i, :L], enc.S[enc.S_ptr[i]:enc.S_ptr[i + 1]])
        assert np.all(S[i, L:] == -1)


# ---- edge cases ---------------------------------------------------------------------

SPECIAL = np.array([0.0, -0.0, 1.0, -1.0, np.inf, -np.inf, np.nan, 26.0, 5e-324], dtype=np.float64)


def random_csr(rng, n_rows, n_cols, max_len, pool):
    lens = rng.integers(0, max_len + 1, n_rows)
    lens = np.minimum(lens, n_cols)
    cols = [np.sort(rng.choice(n_cols, size=L, replace=False)) for L in lens]
    rp = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(lens, out=rp[1:])
    col = np.concatenate(cols).astype(np.int32) if n_rows else np.zeros(0, np.int32)
    val = rng.choice(pool, size=int(rp[-1]))
    return CSR(n_rows, n_cols, rp, col, val)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("fmt", FORMATS)
def test_random_special_values_roundtrip_and_spmv(seed, fmt):
    say("case: random special", seed, fmt)
    rng = np.random.default_rng(seed)
    nan_payload = np.frombuffer(np.uint64(0x7FF0000000000777).tobytes(), dtype=np.float64)[0]
    pool = np.concatenate([SPECIAL, [nan_payload], rng.uniform(-5, 5, 4)])
    A = random_csr(rng, int(rng.integers(1, 700)), int(rng.integers(1, 900)), 40, pool)
    M = compress(A, fmt=fmt, min_pattern_rows=1 + seed % 2)
    assert roundtrip_ok(M, A)
    x = rng.uniform(-1, 1, A.n_cols)
    y = gpu_spmv(M, x)
    yref = oracle.spmv(A, x)
    # special values: NaN where the oracle has NaN, otherwise the 1e-14 bound
    nan = np.isnan(yref)
    assert np.array_equal(np.isnan(y), nan)
    fin = ~nan & np.isfinite(yref)
    s = row_scale(A, x)[fin]
    assert np.all(np.abs(y[fin] - yref[fin]) <= 1e-14 * s + 0.0)
    inf = ~nan & ~np.isfinite(yref)
    assert np.array_equal(y[inf], yref[inf])


@pytest.mark.parametrize("fmt", FORMATS)
def test_long_rows_escape_and_empty_rows(fmt):
    say("case: long rows", fmt)
    rng = np.random.default_rng(9)
    n_rows, n_cols = 300, 1000
    lens = np.zeros(n_rows, dtype=np.int64)
    lens[5] = 600  # longer than 255: escape row
    lens[100:200] = 7
    cols = [np.sort(rng.choice(n_cols, size=L, replace=False)) for L in lens]
    rp = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(lens, out=rp[1:])
    A = CSR(n_rows, n_cols, rp, np.concatenate(cols).astype(np.int32), rng.choice([-1.0, 2.0, 0.5], int(rp[-1])))
    M = compress(A, fmt=fmt)
    assert roundtrip_ok(M, A)
    x = rng.uniform(-1, 1, n_cols)
    assert max_rel_err(A, x, gpu_spmv(M, x), oracle.spmv(A, x)) <= 1e-14
    assert M.info()["n_escape_rows"] >= 1


def test_empty_matrix_and_single_row():
    say("case: empty / single row")
    torch = torch_mod()
    P = lib()
    A = CSR(3, 5, np.zeros(4, dtype=np.int64), np.zeros(0, np.int32), np.zeros(0))
    for fmt in FORMATS:  # every row empty
        M = P.compress(torch.zeros(4, dtype=torch.int64, device="cuda"), torch.zeros(0, dtype=torch.int32, device="cuda"),
                       torch.zeros(0, dtype=torch.float64, device="cuda"), n_cols=5, fmt=fmt)
        y = M.spmv(torch.ones(5, dtype=torch.float64, device="cuda"))
        assert torch.all(y == 0)
        assert roundtrip_ok(M, A)
    for fmt in ("DIT", "DITV"):  # no rows at all
        M = P.compress(torch.zeros(1, dtype=torch.int64, device="cuda"), torch.zeros(0, dtype=torch.int32, device="cuda"),
                       torch.zeros(0, dtype=torch.float64, device="cuda"), n_cols=4, fmt=fmt)
        assert M.spmv(torch.ones(4, dtype=torch.float64, device="cuda")).numel() == 0
    B = CSR(1, 66, [0, 5], [45, 49, 50, 51, 65], [-1.0, -1.0, 26.0, -1.0, -1.0])
    for fmt in FORMATS:
        M = compress(B, fmt=fmt, min_pattern_rows=1)
        assert roundtrip_ok(M, B)
        x = uniform_vector(66, seed=2)
        assert max_rel_err(B, x, gpu_spmv(M, x), oracle.spmv(B, x)) <= 1e-14


def test_invalid_csr_is_rejected():
    say("case: invalid CSR")
    torch = torch_mod()
    P = lib()
    dev = "cuda"
    rp = torch.tensor([0, 2, 3], dtype=torch.int64, device=dev)
    with pytest.raises(P.SpmvcError) as e:  # unsorted columns
        P.compress(rp, torch.tensor([3, 1, 0], dtype=torch.int32, device=dev),
                   torch.ones(3, dtype=torch.float64, device=dev), n_cols=4)
    assert e.value.status == -3
    with pytest.raises(P.SpmvcError) as e:  # column out of range
        P.compress(rp, torch.tensor([1, 9, 0], dtype=torch.int32, device=dev),
                   torch.ones(3, dtype=torch.float64, device=dev), n_cols=4)
    assert e.value.status == -4
    with pytest.raises(P.SpmvcError) as e:  # row_ptr not ending at nnz
        P.compress(torch.tensor([0, 2, 5], dtype=torch.int64, device=dev),
                   torch.tensor([0, 1, 2], dtype=torch.int32, device=dev),
                   torch.ones(3, dtype=torch.float64, device=dev), n_cols=4)
    assert e.value.status == -4
    A = stencil27(4, 4, 4)
    M = compress(A)
    x = torch.ones(A.n_cols, dtype=torch.float64, device=dev)
    with pytest.raises(P.SpmvcError) as e:  # x and y alias
        M.spmv(x, x)
    assert e.value.status == -1


def test_torch_allocator_hooks():
    """spmvc_set_allocator: with torch's caching allocator installed, compression,
    SpMV, block SpMV, CG and SymGS allocate through it (counted here) and give
    the oracle's results; handles made under it are freed back to it after the
    hooks are removed again."""
    say("case: allocator hooks")
    torch = torch_mod()
    P = lib()
    import ctypes

    counts = {"alloc": 0, "free": 0}
    alloc_t = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
    free_t = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)

    def _alloc(n, s, c):
        counts["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(int(n))

    def _free(p, s, c):
        counts["free"] += 1
        torch.cuda.caching_allocator_delete(p)

    hooks = (alloc_t(_alloc), free_t(_free))
    P._alloc_hooks.append(hooks)  # kept alive for as long as buffers made with them may exist
    assert P.load().spmvc_set_allocator(hooks[0], hooks[1], None) == 0
    try:
        A = stencil27(20, 18, 16)
        x = uniform_vector(A.n_cols, seed=31)
        for fmt in ("DIT", "DITV", "ELL"):
            M = compress(A, fmt=fmt)
            assert max_rel_err(A, x, gpu_spmv(M, x), oracle.spmv(A, x)) <= 1e-14
            X = np.stack([uniform_vector(A.n_cols, seed=40 + r) for r in range(8)], axis=1)
            Y = M.spmv_block(torch.from_numpy(X).cuda()).cpu().numpy()
            Yref = oracle.spmv_block(A, X)
            assert all(max_rel_err(A, X[:, r], Y[:, r], Yref[:, r]) <= 1e-14 for r in range(8))
        b = oracle.spmv(A, np.ones(A.n_cols))
        st, xs, stats = P.cg_solve(M, torch.from_numpy(b).cuda())
        torch.cuda.synchronize()
        assert st == 0 and oracle.relres(A, b, xs[0].cpu().numpy()) <= 1e-10
        Mg = compress(A, fmt="DIT")
        xg = Mg.symgs(torch.from_numpy(b).cuda())
        torch.cuda.synchronize()
        assert np.all(np.isfinite(xg.cpu().numpy()))
        assert counts["alloc"] > 0 and counts["free"] > 0
    finally:
        P.use_torch_allocator(False)
    n_alloc = counts["alloc"]
    del M, Mg
    import gc

    gc.collect()
    torch.cuda.synchronize()
    assert counts["alloc"] == n_alloc  # nothing new after the hooks were removed
    assert counts["free"] == counts["alloc"]  # every buffer went back to the hooks that made it
    # and plain hipMalloc again afterwards
    M2 = compress(A, fmt="DIT")
    assert max_rel_err(A, x, gpu_spmv(M2, x), oracle.spmv(A, x)) <= 1e-14
    assert counts["alloc"] == n_alloc


def test_auto_format_choice():
    """fmt=AUTO keeps DIT for the stencil (3 B/row against ELL's 324) and falls
    back to ELL where every row's pattern is unique (all rows would escape as
    CSR, more bytes than ELL's 12 per slot); both multiply correctly."""
    say("case: AUTO format")
    A = stencil27(16, 16, 16)
    M = compress(A, fmt="AUTO")
    assert M.info()["fmt_name"] == "DIT"
    x = uniform_vector(A.n_cols, seed=33)
    assert max_rel_err(A, x, gpu_spmv(M, x), oracle.spmv(A, x)) <= 1e-14
    rng = np.random.default_rng(34)
    n, L = 500, 8
    cols = np.concatenate([np.sort(rng.choice(2000, L, replace=False)) for _ in range(n)]).astype(np.int32)
    B = CSR(n, 2000, np.arange(0, n * L + 1, L, dtype=np.int64), cols, rng.choice([-1.0, 2.0], n * L))
    Mb = compress(B, fmt="AUTO")
    assert Mb.info()["fmt_name"] == "ELL"
    xb = uniform_vector(B.n_cols, seed=35)
    assert max_rel_err(B, xb, gpu_spmv(Mb, xb), oracle.spmv(B, xb)) <= 1e-14
    assert roundtrip_ok(Mb, B)
