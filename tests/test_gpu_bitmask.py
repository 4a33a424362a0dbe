"""GPU neighbour-bitmask format (BMASK) against the oracle, through the C ABI.

* the encoded arrays (displacement list D, row masks, V[1] masks, values)
  equal the oracle's encoding (oracle/bitmask.py), up to the full irregular
  128^3 matrix, and decompression is bit-exact;
* FP64 SpMV within 1e-14 of the oracle per row (relative to sum |a||x|), FP32
  within (len + 2) 2^-24 of it, in every kernel configuration (LDS windows
  at 256, 512 and 1024 rows per block, the direct gather) and the tuned one;
* block SpMV, CG (every mode and the allocation-free entry point) and SymGS
  take BMASK matrices like any other format.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import bitmask as bm
from oracle import gs
from synthetic import CSR, stencil27, stencil27_irregular, uniform_vector

from gpu_util import compress, lib, max_rel_err, same_bits, torch_mod

pytestmark = pytest.mark.gpu

CONFIGS = [(256, 1), (512, 1), (1024, 1), (512, 0)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _np(t, dtype):
    return t.cpu().numpy().view(dtype)


def _three_values():
    A = stencil27(11, 9, 8)
    A.val[::7] = 3.5  # three distinct values: no table
    return A


def _one_value():
    A = stencil27(9, 8, 7)
    A.val[:] = 2.0
    return A


def _wide_rows():
    """33 displacements: 8-byte masks; some rows empty."""
    n = 300
    rng = np.random.default_rng(3)
    rp, cols = [0], []
    for i in range(n):
        if i % 5 != 4:
            cols += [j for j in range(i - 16, i + 17) if 0 <= j < n and (j == i or rng.random() < 0.7)]
        rp.append(len(cols))
    return CSR(n, n, np.array(rp), np.array(cols, dtype=np.int32), rng.uniform(-1, 1, len(cols)))


MAKERS = {
    "stencil16": lambda: stencil27(16, 16, 16),
    "stencil7x5x3": lambda: stencil27(7, 5, 3),
    "irregular": lambda: stencil27_irregular(20, 17, 13, seed=1),
    "three_values": _three_values,
    "one_value": _one_value,
    "wide_rows": _wide_rows,
    "irregular128": lambda: stencil27_irregular(128, 128, 128, seed=0),
}


@pytest.mark.parametrize("name", list(MAKERS))
def test_arrays_equal_oracle_and_roundtrip(name):
    say("case: bmask arrays", name)
    A = MAKERS[name]()
    enc = bm.encode_bitmask(A)
    M = compress(A, fmt="BMASK")
    inf = M.info()
    n = A.n_rows
    assert inf["fmt_name"] == "BMASK" and inf["P"] == enc.D.size and inf["id_bytes"] == enc.mask_bytes
    assert inf["K"] == enc.K and same_bits(np.array(inf["V"]), enc.V)
    assert inf["n_escape_rows"] == 0
    assert np.array_equal(_np(M.array("BM_D"), np.int32).astype(np.int64), enc.D)
    mt = np.uint32 if enc.mask_bytes == 4 else np.uint64
    assert np.array_equal(_np(M.array("BM_MASK"), mt)[:n].astype(np.uint64), enc.mask)
    if enc.K == 2:
        assert np.array_equal(_np(M.array("BM_VMASK"), mt)[:n].astype(np.uint64), enc.vmask)
    else:
        assert M.array("BM_VMASK").numel() == 0
    if enc.K == 0:  # values of every row in column order, slices of 64 rows
        raw = _np(M.array("RAW"), np.float64)
        sl = _np(M.array("RAW_SLICE"), np.int64)
        k = np.diff(enc.raw_ptr)
        rows = np.repeat(np.arange(n, dtype=np.int64), k)
        j = np.arange(enc.raw.size, dtype=np.int64) - enc.raw_ptr[rows]
        assert same_bits(raw[sl[rows // 64] + rows % 64 + 64 * j], enc.raw)
    rp, col, val = M.decompress()
    assert np.array_equal(rp.cpu().numpy(), A.row_ptr) and np.array_equal(col.cpu().numpy(), A.col)
    assert same_bits(val.cpu().numpy(), A.val)


@pytest.mark.parametrize("name", ["stencil16", "irregular", "three_values", "one_value", "wide_rows",
                                  "stencil104", "irregular128"])
def test_spmv_every_configuration(name):
    say("case: bmask spmv", name)
    torch = torch_mod()
    A = stencil27(104, 104, 104) if name == "stencil104" else MAKERS[name]()
    x = uniform_vector(A.n_cols, seed=8)
    yref = oracle.spmv(A, x)
    x32 = x.astype(np.float32)
    y32ref = oracle.spmv(A, x32.astype(np.float64))
    absA = CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, np.abs(A.val))
    s32 = oracle.spmv(absA, np.abs(x32.astype(np.float64)))
    lens = np.diff(A.row_ptr)
    M = compress(A, fmt="BMASK")
    xt, xt32 = torch.from_numpy(x).cuda(), torch.from_numpy(x32).cuda()
    for rows, lds in CONFIGS + [(None, None)]:
        if rows is None:
            M.tune(torch.float64)
            M.tune(torch.float32)
        else:
            M.set_config(rows, lds)
        inf = M.info()
        say("  config", rows, lds, inf["kernel_name"], inf["kernel_name_f32"])
        if lds == 1:
            assert inf["kernel_name"] == "k_bmask_lds"
        y = M.spmv(xt).cpu().numpy()
        assert max_rel_err(A, x, y, yref) <= 1e-14, (rows, lds)
        y32 = M.spmv(xt32).double().cpu().numpy()
        assert np.all(np.abs(y32 - y32ref) <= (lens + 2) * 2.0 ** -24 * s32 + 1e-300), (rows, lds)
    # closed form for the stencil: A*1 = 26 - #neighbours, exact in any order
    if name in ("stencil16", "stencil104"):
        y1 = M.spmv(torch.ones(A.n_cols, dtype=torch.float64, device="cuda")).cpu().numpy()
        assert np.array_equal(y1, oracle.spmv(A, np.ones(A.n_cols)))


def test_x_not_16_byte_aligned():
    """x one element into its buffer: the windows are copied through registers."""
    torch = torch_mod()
    A = stencil27_irregular(24, 20, 18, seed=2)
    x = uniform_vector(A.n_cols, seed=9)
    M = compress(A, fmt="BMASK")
    buf = torch.zeros(A.n_cols + 1, dtype=torch.float64, device="cuda")
    buf[1:] = torch.from_numpy(x).cuda()
    for rows in (256, 512, 1024):
        M.set_config(rows, 1)
        y = M.spmv(buf[1:]).cpu().numpy()
        assert max_rel_err(A, x, y, oracle.spmv(A, x)) <= 1e-14


@pytest.mark.parametrize("nrhs", [1, 3, 8, 16])
def test_block_spmv(nrhs):
    say("case: bmask block", nrhs)
    torch = torch_mod()
    for A in (stencil27(21, 18, 15), stencil27_irregular(20, 18, 15, seed=4)):
        X = np.stack([uniform_vector(A.n_cols, seed=20 + r) for r in range(nrhs)], axis=1)
        M = compress(A, fmt="BMASK")
        Y = M.spmv_block(torch.from_numpy(X).cuda()).cpu().numpy()
        Yref = oracle.spmv_block(A, X)
        for r in range(nrhs):
            assert max_rel_err(A, X[:, r], Y[:, r], Yref[:, r]) <= 1e-14


def test_cg_every_mode():
    """FP64, mixed precision, SymGS-preconditioned, batched pairs (solved one
    after another: the batched kernels take DIT) and the allocation-free entry
    point all reach 1e-10 in the oracle's residual on a BMASK matrix."""
    say("case: bmask cg")
    torch = torch_mod()
    P = lib()
    A = stencil27(24, 22, 20)
    b = oracle.spmv(A, np.ones(A.n_cols))
    M = compress(A, fmt="BMASK")
    bt = torch.from_numpy(b).cuda()
    _, _, it_ref, _ = oracle.cg(A, b)
    for mode in (0, 1, 2):
        st, xs, stats = P.cg_solve(M, bt, mode=mode)
        torch.cuda.synchronize()
        x = xs[0].cpu().numpy()
        assert st == 0 and oracle.relres(A, b, x) <= 1e-10, (mode, st)
        if mode == 0:
            assert abs(stats[0]["iters"] - it_ref) <= 2
    st, x, stats = P.cg_solve_noalloc(M, bt)
    torch.cuda.synchronize()
    assert st == 0 and oracle.relres(A, b, x.cpu().numpy()) <= 1e-10
    B = np.stack([uniform_vector(A.n_rows, seed=30 + r) for r in range(3)], axis=1)
    st, xs, stats = P.cg_solve([M], [torch.from_numpy(B).cuda()], nrhs=3)
    torch.cuda.synchronize()
    assert st == 0
    assert P.batched_config()["form"] == -2  # reported: solved one pair after another
    X = xs[0].cpu().numpy()
    for r in range(3):
        assert oracle.relres(A, B[:, r], X[:, r]) <= 1e-10


def test_symgs_equals_oracle():
    say("case: bmask symgs")
    torch = torch_mod()
    for A in (stencil27(12, 10, 9), stencil27_irregular(10, 9, 8, seed=3)):
        b = uniform_vector(A.n_rows, seed=5)
        x0 = uniform_vector(A.n_rows, seed=6)
        M = compress(A, fmt="BMASK")
        nc, col = M.colors()
        color = gs.greedy_coloring(A)
        assert np.array_equal(col.cpu().numpy().astype(np.int64), color)
        x = torch.from_numpy(x0.copy()).cuda()
        M.symgs(torch.from_numpy(b).cuda(), x, sweeps=2)
        torch.cuda.synchronize()
        ref = gs.symgs(A, b, x0, color, sweeps=2)
        scale = max(1.0, float(np.abs(ref).max()), float(np.abs(b).max()))
        assert float(np.abs(x.cpu().numpy() - ref).max()) <= 1e-12 * scale


def test_limits_and_degenerate_matrices():
    """65 displacements are refused (SPMVC_EUNSUPPORTED); an empty matrix, a
    matrix without entries and a single row compress and multiply."""
    say("case: bmask limits")
    torch = torch_mod()
    P = lib()
    n = 80
    cols = np.arange(65, dtype=np.int32)
    A = CSR(n, n, np.concatenate([[0], np.full(n, 65)]), cols, np.ones(65))
    with pytest.raises(P.SpmvcError) as e:
        compress(A, fmt="BMASK")
    assert e.value.status == -8
    for A in (CSR(0, 0, np.zeros(1, dtype=np.int64), np.zeros(0, dtype=np.int32), np.zeros(0)),
              CSR(5, 5, np.zeros(6, dtype=np.int64), np.zeros(0, dtype=np.int32), np.zeros(0)),
              CSR(1, 7, np.array([0, 3]), np.array([1, 4, 6], dtype=np.int32), np.array([1.0, -2.0, 0.5]))):
        M = compress(A, fmt="BMASK")
        x = uniform_vector(A.n_cols, seed=1)
        if A.n_rows:
            y = M.spmv(torch.from_numpy(x).cuda()).cpu().numpy()
            assert np.array_equal(y, oracle.spmv(A, x))
        rp, col, val = M.decompress()
        assert np.array_equal(rp.cpu().numpy(), A.row_ptr) and np.array_equal(col.cpu().numpy(), A.col)
