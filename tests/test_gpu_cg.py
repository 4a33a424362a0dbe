"""GPU conjugate gradients against the CPU oracle.

The result of every solve is checked with the oracle's FP64 SpMV: the true
relative residual ||b - A x|| / ||b|| must be <= 1e-10 (plus a little slack
for the final rounding), and for b = A*1 the solution must approach 1.
Iteration counts of the FP64 solver must match the oracle's within 2 (the
two sum in different orders).
"""
import sys

import numpy as np
import pytest

import oracle
from synthetic import CSR, batched_grids, stencil27, stencil27_irregular, stencil_hierarchy, uniform_vector

from gpu_util import compress, lib, torch_mod

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def solve(A, b, fmt="DIT", **kw):
    torch = torch_mod()
    P = lib()
    M = compress(A, fmt=fmt)
    bt = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    st, xs, stats = P.cg_solve(M, bt, **kw)
    torch.cuda.synchronize()
    return st, xs[0].cpu().numpy(), stats


@pytest.mark.parametrize("fmt", ["ELL", "DT", "DIT", "DITV"])
@pytest.mark.parametrize("grid", [(16, 16, 16), (32, 32, 32)])
def test_fp64_cg_ones(fmt, grid):
    say("case: cg ones", fmt, grid)
    A = stencil27(*grid)
    b = oracle.spmv(A, np.ones(A.n_cols))
    st, x, stats = solve(A, b, fmt=fmt)
    _, _, it_ref, _ = oracle.cg(A, b)
    assert st == 0 and stats[0]["status"] == 0
    assert abs(stats[0]["iters"] - it_ref) <= 2
    assert oracle.relres(A, b, x) <= 1e-10
    assert abs(stats[0]["relres_true"] - oracle.relres(A, b, x)) <= 1e-12
    assert np.abs(x - 1).max() < 1e-7


@pytest.mark.parametrize("rows,lds", [(256, 2), (512, 2), (1024, 1), (512, 0)])
def test_cg_under_each_spmv_configuration(rows, lds):
    """CG takes its p.Ap partials from whichever SpMV kernel the handle runs
    (plane-marching, register, direct gather), with that kernel's own number of
    blocks; FP64 and mixed precision must still reach the oracle's result."""
    say("case: cg config", rows, lds)
    torch = torch_mod()
    P = lib()
    A = stencil27(48, 40, 36)
    b = oracle.spmv(A, np.ones(A.n_cols))
    M = compress(A, fmt="DIT")
    M.set_config(rows, lds)
    bt = torch.from_numpy(b).cuda()
    _, _, it_ref, _ = oracle.cg(A, b)
    for mode in (0, 1):
        st, xs, stats = P.cg_solve(M, bt, mode=mode)
        torch.cuda.synchronize()
        x = xs[0].cpu().numpy()
        assert st == 0 and stats[0]["status"] == 0
        if mode == 0:
            assert abs(stats[0]["iters"] - it_ref) <= 2
        assert oracle.relres(A, b, x) <= 1e-10
        assert np.abs(x - 1).max() < 1e-7


@pytest.mark.parametrize("offset", [0, 1])
def test_cg_odd_size_and_unaligned_vectors(offset):
    """The CG update kernels move 16-byte packs when every vector they touch is
    16-byte aligned and handle the last n mod 2 (FP64) or n mod 4 (FP32)
    elements one at a time; with x and b one element into their buffers the
    x/p update falls back to 8-byte accesses.  Both must give the oracle's
    solve, in FP64 and mixed precision, on a grid whose n = 7*9*11 is odd."""
    say("case: cg odd/unaligned", offset)
    torch = torch_mod()
    P = lib()
    A = stencil27(7, 9, 11)
    b = oracle.spmv(A, np.ones(A.n_cols))
    M = compress(A, fmt="DIT")
    _, _, it_ref, _ = oracle.cg(A, b)
    bbuf = torch.zeros(A.n_rows + 1, dtype=torch.float64, device="cuda")
    bbuf[offset:offset + A.n_rows] = torch.from_numpy(b).cuda()
    bt = bbuf[offset:offset + A.n_rows]
    for mode in (0, 1):
        xbuf = torch.full((A.n_rows + 1,), 7.0, dtype=torch.float64, device="cuda")
        xt = xbuf[offset:offset + A.n_rows]
        st, _, stats = P.cg_solve(M, bt, xs=xt, mode=mode)
        torch.cuda.synchronize()
        x = xt.cpu().numpy()
        assert st == 0 and stats[0]["status"] == 0
        if mode == 0:
            assert abs(stats[0]["iters"] - it_ref) <= 2
        assert oracle.relres(A, b, x) <= 1e-10
        assert np.abs(x - 1).max() < 1e-7
        rest = xbuf.cpu().numpy()
        assert rest[0 if offset else A.n_rows] == 7.0  # the element outside the view is untouched


def test_cg_full_size_192():
    """The 192^3 stencil (7.08 M rows, 189 M nnz) with b = A*1, in the launch
    configuration the benchmark times (FP64 and FP32 SpMV tuned): the FP64
    solve takes the oracle's iteration count within 2, and FP64 and mixed
    precision both reach 1e-10 in the oracle's own residual with x close to 1."""
    say("case: cg full size 192^3")
    torch = torch_mod()
    P = lib()
    A = stencil27(192, 192, 192)
    b = oracle.spmv(A, np.ones(A.n_cols))
    M = compress(A, fmt="DIT")
    M.tune(torch.float64)
    M.tune(torch.float32)
    bt = torch.from_numpy(b).cuda()
    say("  oracle cg")
    _, st_ref, it_ref, _ = oracle.cg(A, b)
    assert st_ref == 0
    for mode in (0, 1, 3):
        say("  gpu cg mode", mode)
        st, xs, stats = P.cg_solve(M, bt, mode=mode, inner_rtol=1e-2 if mode == 3 else 1e-5)
        torch.cuda.synchronize()
        x = xs[0].cpu().numpy()
        say("  ", stats[0])
        assert st == 0 and stats[0]["status"] == 0
        if mode == 0:
            assert abs(stats[0]["iters"] - it_ref) <= 2
        if mode == 3:  # the Krylov space survives the replacements
            assert stats[0]["iters"] <= 1.3 * it_ref
        assert oracle.relres(A, b, x) <= 1e-10
        assert np.abs(x - 1).max() < 1e-6


def test_fp64_cg_random_rhs_irregular():
    say("case: cg irregular")
    A = stencil27_irregular(30, 28, 26, seed=0)
    b = uniform_vector(A.n_rows, seed=0)
    st, x, stats = solve(A, b)
    _, _, it_ref, _ = oracle.cg(A, b)
    assert st == 0 and abs(stats[0]["iters"] - it_ref) <= 2
    assert oracle.relres(A, b, x) <= 1e-10


@pytest.mark.parametrize("grid", [(16, 16, 16), (64, 64, 64)])
def test_mixed_precision_reaches_fp64_tolerance(grid):
    say("case: mixed", grid)
    A = stencil27(*grid)
    b = oracle.spmv(A, np.ones(A.n_cols))
    st, x, stats = solve(A, b, mode=1)
    assert st == 0
    assert stats[0]["outer_iters"] >= 1
    assert oracle.relres(A, b, x) <= 1e-10
    assert np.abs(x - 1).max() < 1e-7


@pytest.mark.parametrize("grid", [(16, 16, 16), (64, 64, 64), (61, 17, 33)])
@pytest.mark.parametrize("delta", [1e-1, 1e-2, 1e-4])
def test_reliable_updates_reach_fp64_tolerance(grid, delta):
    """Mode 3 (FP32 CG with the FP64 residual put back every time the
    recursive one falls by delta): the oracle's true residual <= 1e-10, x
    close to 1, more than one segment, and at most 1.4 times the FP64
    iteration count: the search direction is kept across replacements, and
    what remains is the slower convergence of CG in FP32 arithmetic (1.26 to
    1.37 times FP64's count at 64^3 to 192^3, against 1.41 for refinement
    restarts at 192^3)."""
    say("case: reliable updates", grid, delta)
    A = stencil27(*grid)
    b = oracle.spmv(A, np.ones(A.n_cols))
    _, _, it_ref, _ = oracle.cg(A, b)
    st, x, stats = solve(A, b, mode=3, inner_rtol=delta)
    say("  ", stats[0], "fp64 iters", it_ref)
    assert st == 0 and stats[0]["status"] == 0
    assert stats[0]["outer_iters"] >= 2
    assert stats[0]["iters"] <= 1.4 * it_ref + 4
    assert oracle.relres(A, b, x) <= 1e-10
    assert abs(stats[0]["relres_true"] - oracle.relres(A, b, x)) <= 1e-13
    assert np.abs(x - 1).max() < 1e-7


def test_reliable_updates_irregular_random_rhs():
    say("case: reliable updates irregular")
    A = stencil27_irregular(30, 28, 26, seed=0)
    b = uniform_vector(A.n_rows, seed=0)
    _, _, it_ref, _ = oracle.cg(A, b)
    for fmt in ("DIT", "BMASK", "ELL"):
        st, x, stats = solve(A, b, fmt=fmt, mode=3, inner_rtol=1e-2)
        assert st == 0 and stats[0]["iters"] <= 1.4 * it_ref + 4, (fmt, stats)
        assert oracle.relres(A, b, x) <= 1e-10


def test_reliable_updates_failures():
    """Breakdown (negative definite), the iteration cap, a zero right-hand side
    and options the mode rejects (several systems, inner_rtol <= 0)."""
    say("case: reliable updates failures")
    torch = torch_mod()
    P = lib()
    A = stencil27(8, 8, 8)
    A.val[:] = -A.val
    st, x, stats = solve(A, np.ones(A.n_rows), mode=3)
    assert st == -6 and stats[0]["iters"] == 1
    B = stencil27(16, 16, 16)
    st, x, stats = solve(B, uniform_vector(B.n_rows, seed=0), mode=3, max_iter=5)
    assert st == -7 and stats[0]["iters"] == 5
    st, x, stats = solve(B, np.zeros(B.n_rows), mode=3)
    assert st == 0 and stats[0]["iters"] == 0 and np.all(x == 0)
    M = compress(B)
    bt = torch.from_numpy(uniform_vector(B.n_rows, seed=1)).cuda()
    st, _, _ = P.cg_solve([M, M], [bt, bt], mode=3)
    assert st == -8
    st, _, _ = P.cg_solve(M, bt, mode=3, inner_rtol=0.0)
    assert st == -1
    st, _, _ = P.cg_solve(M, bt, mode=4)
    assert st == -1


def test_reliable_updates_replacement_cap():
    """max_outer caps the replacements (decided on the device between
    segments): with max_outer = k the solve stops with SPMVC_ENOCONV after
    k + 1 segments; the reported true residual is the oracle's residual of
    the returned x, the recursive one that of the last segment (close to it),
    and both fall as k grows."""
    say("case: reliable updates replacement cap")
    A = stencil27(24, 20, 16)
    b = oracle.spmv(A, np.ones(A.n_cols))
    prev_rel, prev_iters = np.inf, 0
    for k in (0, 1, 2):
        st, x, stats = solve(A, b, mode=3, inner_rtol=1e-2, max_outer=k)
        s = stats[0]
        say("  ", k, s)
        rel = oracle.relres(A, b, x)
        assert st == -7 and s["status"] == -7 and s["outer_iters"] == k + 1
        assert rel > 1e-10 and rel < prev_rel and s["iters"] > prev_iters
        assert abs(s["relres_true"] - rel) <= 1e-12
        assert 0.5 * rel <= s["relres_recursive"] <= 2.0 * rel
        prev_rel, prev_iters = rel, s["iters"]
    st, x, stats = solve(A, b, mode=3, inner_rtol=1e-2)
    assert st == 0 and stats[0]["outer_iters"] >= 3 and oracle.relres(A, b, x) <= 1e-10


@pytest.mark.parametrize("scale", [1e-36, 1e39])
def test_mixed_precision_scaled_rhs(scale):
    """b = scale * A*1 with scale outside the FP32 range of the residual
    (1e-36: its square underflows in FP32; 1e39: it overflows): the FP32 inner
    solve takes r / ||r||, so mixed precision reaches 1e-10 as FP64 does, with
    x = scale * 1."""
    say("case: mixed scaled rhs", scale)
    A = stencil27(24, 20, 18)
    b = oracle.spmv(A, np.full(A.n_cols, scale))
    for mode in (0, 1, 3):
        st, x, stats = solve(A, b, mode=mode)
        assert st == 0 and stats[0]["status"] == 0, (mode, stats)
        assert oracle.relres(A, b, x) <= 1e-10
        assert np.abs(x / scale - 1).max() < 1e-7


@pytest.mark.parametrize("rtol", [1e-12, 1e-15, 1e-17])
def test_true_residual_guarantee(rtol):
    """A solve reports SPMVC_OK only when its own true FP64 residual meets the
    tolerance, else SPMVC_ENOCONV with the true residual it reached: near the
    FP64 floor (1e-15) the recursive residual can pass first, and the solver
    restarts from b - A x; at 1e-17 (below the rounding of b - A x itself)
    every solve must end SPMVC_ENOCONV, never with a false OK.  Single FP64,
    SymGS-preconditioned, and batched pairs."""
    say("case: true residual guarantee", rtol)
    torch = torch_mod()
    P = lib()
    A = stencil27(20, 18, 16)
    b = uniform_vector(A.n_rows, seed=4)
    M = compress(A)
    runs = []
    for mode in (0, 2):
        st, xs, stats = P.cg_solve(M, torch.from_numpy(b).cuda(), rtol=rtol, mode=mode, max_iter=3000)
        torch.cuda.synchronize()
        runs.append((st, stats[0], xs[0].cpu().numpy(), b))
    B = np.stack([uniform_vector(A.n_rows, seed=40 + r) for r in range(4)], axis=1)
    st, xs, stats = P.cg_solve([M, M], [torch.from_numpy(B).cuda()] * 2, nrhs=4, rtol=rtol, max_iter=3000)
    torch.cuda.synchronize()
    for q, s_ in enumerate(stats):
        runs.append((s_["status"], s_, xs[q // 4].cpu().numpy()[:, q % 4], B[:, q % 4]))
    for st, s_, x, bb in runs:
        rel = oracle.relres(A, bb, x)
        assert abs(s_["relres_true"] - rel) <= 1e-13
        if rtol == 1e-12:
            assert st == 0
        if rtol == 1e-17:
            assert st == -7
        if st == 0:
            assert s_["relres_true"] <= rtol and rel <= rtol + 1e-13
        else:
            assert st == -7 and s_["relres_true"] > rtol


def test_error_paths():
    """Bad arguments the C ABI rejects: nrhs 0 or 17 and leading dimensions
    below nrhs (spmv_block, cg_solve), duplicate columns in a CSR row
    (compression), NaN in b (every CG mode and the batched pairs)."""
    say("case: error paths")
    import ctypes

    torch = torch_mod()
    P = lib()
    L = P.load()
    A = stencil27(8, 8, 8)
    M = compress(A)
    X = torch.zeros((A.n_cols, 16), dtype=torch.float64, device="cuda")
    Y = torch.zeros((A.n_rows, 16), dtype=torch.float64, device="cuda")
    px, py = ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr())
    for nrhs, ldx, ldy in [(0, 16, 16), (17, 17, 17), (8, 4, 16), (8, 16, 7)]:
        assert L.spmv_block(M.handle, 0, nrhs, px, ldx, py, ldy, None) == -1, (nrhs, ldx, ldy)
    b = torch.ones(A.n_rows * 17, dtype=torch.float64, device="cuda")
    for nrhs in (0, 17):
        st, _, _ = P.cg_solve([M], [b], nrhs=nrhs)
        assert st == -1, nrhs
    dev = "cuda"
    with pytest.raises(P.SpmvcError) as e:  # a column repeated within a row
        P.compress(torch.tensor([0, 3, 4], dtype=torch.int64, device=dev),
                   torch.tensor([0, 2, 2, 1], dtype=torch.int32, device=dev),
                   torch.ones(4, dtype=torch.float64, device=dev), n_cols=4)
    assert e.value.status == -3
    bn = oracle.spmv(A, np.ones(A.n_cols))
    bn[17] = np.nan
    for mode in (0, 1, 2, 3):
        st, x, stats = solve(A, bn, mode=mode)
        assert st == -1 and stats[0]["status"] == -1, (mode, st, stats)
    B = np.stack([oracle.spmv(A, np.ones(A.n_cols))] * 2, axis=1)
    B[5, 1] = np.nan
    st, xs, stats = P.cg_solve([M], [torch.from_numpy(B).cuda()], nrhs=2)
    torch.cuda.synchronize()
    assert st == -1 and stats[0]["status"] == 0 and stats[1]["status"] == -1
    assert oracle.relres(A, B[:, 0], xs[0].cpu().numpy()[:, 0]) <= 1e-10


def test_multi_rhs_and_systems():
    say("case: multi rhs")
    torch = torch_mod()
    P = lib()
    grids = [(10, 12, 9), (16, 11, 13)]
    mats, As, bs = [], [], []
    for g in grids:
        A = stencil27(*g)
        As.append(A)
        mats.append(compress(A))
        B = np.stack([uniform_vector(A.n_rows, seed=s) for s in range(3)], axis=1)
        bs.append(torch.from_numpy(B).cuda())
    st, xs, stats = P.cg_solve(mats, bs, nrhs=3)
    torch.cuda.synchronize()
    assert st == 0
    for s, A in enumerate(As):
        X = xs[s].cpu().numpy()
        B = bs[s].cpu().numpy()
        for r in range(3):
            assert oracle.relres(A, B[:, r], X[:, r]) <= 1e-10
            assert stats[s * 3 + r]["status"] == 0


def test_breakdown_and_max_iter():
    say("case: cg failures")
    A = stencil27(8, 8, 8)
    A.val[:] = -A.val  # negative definite: p.Ap < 0 at the first step
    st, x, stats = solve(A, np.ones(A.n_rows))
    assert st == -6 and stats[0]["iters"] == 1
    B = stencil27(16, 16, 16)
    st, x, stats = solve(B, uniform_vector(B.n_rows, seed=0), max_iter=5)
    assert st == -7 and stats[0]["iters"] == 5


def test_zero_rhs():
    say("case: zero rhs")
    A = stencil27(8, 8, 8)
    st, x, stats = solve(A, np.zeros(A.n_rows))
    assert st == 0 and stats[0]["iters"] == 0 and np.all(x == 0)


# ---- batched CG: uneven systems x several right-hand sides ---------------------------

def batched_case(grids, nrhs, seed=0):
    torch = torch_mod()
    mats, As, bs = [], [], []
    rng = np.random.default_rng(seed)
    for g in grids:
        A = stencil27(*g)
        As.append(A)
        mats.append(compress(A))
        B = rng.uniform(-1, 1, (A.n_rows, nrhs))
        bs.append(torch.from_numpy(B).cuda())
    return mats, As, bs


@pytest.mark.parametrize("batched", [1, 2])
def test_batched_matches_oracle(batched):
    say("case: batched", batched)
    torch = torch_mod()
    P = lib()
    grids = [(10, 12, 9), (16, 11, 13), (20, 7, 5), (3, 3, 3)]
    mats, As, bs = batched_case(grids, 8)
    st, xs, stats = P.cg_solve(mats, bs, nrhs=8, batched=batched, check_every=5)
    torch.cuda.synchronize()
    assert st == 0
    for s, A in enumerate(As):
        X = xs[s].cpu().numpy()
        B = bs[s].cpu().numpy()
        for r in range(8):
            assert stats[s * 8 + r]["status"] == 0
            assert oracle.relres(A, B[:, r], X[:, r]) <= 1e-10
            _, _, it_ref, _ = oracle.cg(A, B[:, r])
            assert abs(stats[s * 8 + r]["iters"] - it_ref) <= 2
            assert abs(stats[s * 8 + r]["relres_true"] - oracle.relres(A, B[:, r], X[:, r])) <= 1e-12


def test_batched_graph_replays_equal_eager():
    """The graph path (many replays of a 3-iteration graph) equals the eager launches bit for bit."""
    say("case: batched graph vs eager")
    torch = torch_mod()
    P = lib()
    grids = [(12, 10, 8), (17, 9, 6)]
    mats, As, bs = batched_case(grids, 5, seed=3)
    _, x_eager, s_eager = P.cg_solve(mats, bs, nrhs=5, batched=1, check_every=3)
    for _ in range(2):  # the graph is recorded and replayed afresh in each call
        _, x_graph, s_graph = P.cg_solve(mats, bs, nrhs=5, batched=2, check_every=3)
        torch.cuda.synchronize()
        for a, b in zip(x_eager, x_graph):
            assert torch.equal(a, b)
        assert [s["iters"] for s in s_eager] == [s["iters"] for s in s_graph]


@pytest.mark.parametrize("nrhs", [2, 4, 8])
def test_batched_window_phased_spmv(nrhs, monkeypatch):
    """Even nrhs of 2, 4 or 8 take the window-phased batched SpMV (each
    system's windows staged whole-row in LDS).  Systems from a single row of
    tiles to several planes, thin and tiny grids; graph replays equal eager
    launches bit for bit, and every pair reaches the oracle's tolerance."""
    say("case: batched window-phased", nrhs)
    torch = torch_mod()
    P = lib()
    monkeypatch.setenv("SPMVC_BATCHED_SPMV", "0,32")
    grids = [(2, 2, 2), (40, 3, 3), (9, 31, 4), (24, 20, 18)]  # 2^3: every row an escape row
    mats, As, bs = batched_case(grids, nrhs, seed=7)
    _, x_eager, s_eager = P.cg_solve(mats, bs, nrhs=nrhs, batched=1, check_every=4)
    st, x_graph, s_graph = P.cg_solve(mats, bs, nrhs=nrhs, batched=2, check_every=4)
    torch.cuda.synchronize()
    assert st == 0 and P.batched_config()["form"] == 0
    for a, b in zip(x_eager, x_graph):
        assert torch.equal(a, b)
    for s, A in enumerate(As):
        X = x_graph[s].cpu().numpy()
        B = bs[s].cpu().numpy()
        for r in range(nrhs):
            assert s_graph[s * nrhs + r]["status"] == 0
            assert oracle.relres(A, B[:, r], X[:, r]) <= 1e-10


def test_batched_full_size_64_systems():
    """The full batched workload: 64 systems with grid sides drawn from 16..96
    (seed 0), 8 right-hand sides each, in the replayed-graph mode the
    benchmark times.  Every one of the 512 pairs reaches 1e-10 in the oracle's
    own residual, and the reported residual agrees with it."""
    say("case: batched full size")
    torch = torch_mod()
    P = lib()
    grids = batched_grids(64, 16, 96, seed=0)
    mats, As, bs = batched_case(grids, 8, seed=5)
    st, xs, stats = P.cg_solve(mats, bs, nrhs=8, batched=2, max_iter=5000)
    torch.cuda.synchronize()
    assert st == 0
    for s, A in enumerate(As):
        X = xs[s].cpu().numpy()
        B = bs[s].cpu().numpy()
        for r in range(8):
            q = stats[s * 8 + r]
            rel = oracle.relres(A, B[:, r], X[:, r])
            assert q["status"] == 0 and rel <= 1e-10
            assert abs(q["relres_true"] - rel) <= 1e-12


@pytest.mark.parametrize("nrhs", [3, 8])
def test_batched_ditv_equals_dit(nrhs):
    """Batched CG over DITV handles (T from the pattern table) gives DIT's
    iterates bit for bit -- through the window-phased SpMV (8 right-hand
    sides) and the lane-group one (3) -- and reaches the oracle's tolerance."""
    say("case: batched DITV", nrhs)
    torch = torch_mod()
    P = lib()
    grids = [(10, 12, 9), (16, 11, 13), (3, 3, 3)]
    mats, As, bs = batched_case(grids, nrhs, seed=9)
    mats_v = [compress(A, fmt="DITV") for A in As]
    _, x_d, s_d = P.cg_solve(mats, bs, nrhs=nrhs, batched=2, check_every=4)
    st, x_v, s_v = P.cg_solve(mats_v, bs, nrhs=nrhs, batched=2, check_every=4)
    torch.cuda.synchronize()
    assert st == 0
    assert [q["iters"] for q in s_v] == [q["iters"] for q in s_d]
    for a, b in zip(x_v, x_d):
        assert torch.equal(a, b)
    for s, A in enumerate(As):
        X = x_v[s].cpu().numpy()
        B = bs[s].cpu().numpy()
        for r in range(nrhs):
            assert oracle.relres(A, B[:, r], X[:, r]) <= 1e-10


@pytest.mark.parametrize("form,chunk", [(0, 8), (0, 128), (1, 32), (2, 8), (2, 128)])
def test_batched_spmv_configurations(form, chunk, monkeypatch):
    """Each batched SpMV configuration the tuner can pick (window-phased, lane
    groups with right-hand-side pairs or singles; 8 to 128 tiles per XCD
    chunk), fixed through SPMVC_BATCHED_SPMV: every pair reaches the oracle's
    tolerance, graph replays equal eager launches, and the configuration is
    the one reported."""
    say("case: batched config", form, chunk)
    torch = torch_mod()
    P = lib()
    monkeypatch.setenv("SPMVC_BATCHED_SPMV", f"{form},{chunk}")
    grids = [(12, 10, 9), (20, 7, 5), (3, 3, 3), (30, 26, 22)]
    mats, As, bs = batched_case(grids, 8, seed=11)
    _, x_e, s_e = P.cg_solve(mats, bs, nrhs=8, batched=1, check_every=4)
    st, x_g, s_g = P.cg_solve(mats, bs, nrhs=8, batched=2, check_every=4)
    torch.cuda.synchronize()
    assert st == 0
    assert P.batched_config()["form"] == form and P.batched_config()["chunk"] == chunk
    for a, b in zip(x_e, x_g):
        assert torch.equal(a, b)
    for s, A in enumerate(As):
        X = x_g[s].cpu().numpy()
        B = bs[s].cpu().numpy()
        for r in range(8):
            assert s_g[s * 8 + r]["status"] == 0
            assert oracle.relres(A, B[:, r], X[:, r]) <= 1e-10


def test_batched_tuner_reports_its_choice(monkeypatch):
    say("case: batched tuner")
    torch = torch_mod()
    P = lib()
    monkeypatch.delenv("SPMVC_BATCHED_SPMV", raising=False)
    grids = [(14, 12, 10), (9, 9, 9)]
    mats, As, bs = batched_case(grids, 4, seed=12)
    st, _, _ = P.cg_solve(mats, bs, nrhs=4, batched=2)
    torch.cuda.synchronize()
    cfg = P.batched_config()
    assert st == 0 and cfg["form"] in (0, 1, 2) and cfg["chunk"] in (8, 32, 128) and cfg["us"] > 0


def test_batched_all_systems_empty():
    """A batch whose systems have no rows returns at once: every pair done, no iteration."""
    say("case: batched empty")
    torch = torch_mod()
    P = lib()
    E = CSR(0, 0, np.zeros(1, dtype=np.int64), np.zeros(0, np.int32), np.zeros(0))
    mats = [compress(E, fmt="DIT"), compress(E, fmt="DIT")]
    bs = [torch.zeros((0, 2), dtype=torch.float64, device="cuda") for _ in mats]
    st, xs, stats = P.cg_solve(mats, bs, nrhs=2, batched=2)
    assert st == 0 and all(q["iters"] == 0 and q["status"] == 0 for q in stats)


def test_batched_failures_are_per_pair():
    say("case: batched failures")
    torch = torch_mod()
    P = lib()
    good = stencil27(8, 7, 6)
    bad = stencil27(6, 6, 6)
    bad.val[:] = -bad.val
    mats = [compress(good), compress(bad)]
    bs = [torch.from_numpy(np.ones((A.n_rows, 2))).cuda() for A in (good, bad)]
    st, xs, stats = P.cg_solve(mats, bs, nrhs=2)
    assert st == -6
    assert [s["status"] for s in stats] == [0, 0, -6, -6]
    st, xs, stats = P.cg_solve([mats[0]], [bs[0]], nrhs=2, max_iter=4)
    assert st == -7 and all(s["iters"] == 4 for s in stats)


@pytest.mark.parametrize("fmt,grid", [("DIT", (24, 22, 20)), ("DITV", (17, 13, 11)), ("ELL", (16, 16, 16)),
                                      ("DIT", (64, 64, 64))])
def test_pcg_symgs_matches_oracle(fmt, grid):
    """CG preconditioned by one multicolor SymGS sweep (mode 2): the oracle's
    preconditioned CG (same coloring, same sweep) takes the same iteration
    count within 2, fewer than plain CG, and both reach 1e-10 in the oracle's
    own residual."""
    say("case: pcg", fmt, grid)
    A = stencil27(*grid)
    b = oracle.spmv(A, np.ones(A.n_cols))
    st, x, stats = solve(A, b, fmt=fmt, mode=2)
    assert st == 0 and stats[0]["status"] == 0
    assert oracle.relres(A, b, x) <= 1e-10
    assert np.abs(x - 1).max() < 1e-7
    if A.n_rows <= 20000:
        from oracle import gs

        _, it_ref, _ = gs.pcg(A, b, gs.greedy_coloring(A))
        assert abs(stats[0]["iters"] - it_ref) <= 2
    _, _, it_cg, _ = oracle.cg(A, b)
    assert stats[0]["iters"] < it_cg


def test_pcg_rejects_missing_diagonal_and_zero_rhs():
    say("case: pcg errors")
    A = stencil27(6, 6, 6)
    keep = np.ones(A.nnz, dtype=bool)
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
    keep[np.flatnonzero((rows == 7) & (A.col == 7))] = False
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows[keep], minlength=A.n_rows))])
    B = CSR(A.n_rows, A.n_cols, rp, A.col[keep], A.val[keep])
    st, _, _ = solve(B, np.ones(B.n_rows), mode=2)
    assert st == -1
    st, x, stats = solve(A, np.zeros(A.n_rows), mode=2)
    assert st == 0 and stats[0]["iters"] == 0 and np.all(x == 0)


def mg_solve(mats, f2c, b, fmt="DIT", **kw):
    torch = torch_mod()
    P = lib()
    Ms = [compress(m, fmt=fmt) for m in mats]
    F = [torch.from_numpy(np.ascontiguousarray(f, dtype=np.int32)).cuda() for f in f2c]
    bt = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    st, x, stat = P.cg_solve_mg(Ms, F, bt, **kw)
    torch.cuda.synchronize()
    return st, x.cpu().numpy(), stat


@pytest.mark.parametrize("fmt,grid,levels", [("DIT", (24, 24, 16), 4), ("DITV", (16, 12, 8), 3),
                                             ("ELL", (16, 16, 16), 4), ("DIT", (20, 14, 18), 2),
                                             ("DIT", (64, 64, 64), 4)])
def test_mg_pcg_matches_oracle(fmt, grid, levels):
    """CG preconditioned by one V-cycle: converges to 1e-10 in the oracle's
    residual, in the oracle's iteration count (within 1), and in fewer
    iterations than the single-sweep preconditioner."""
    from oracle import gs

    say("case: mg pcg", fmt, grid, levels)
    mats, f2c = stencil_hierarchy(*grid, levels)
    A = mats[0]
    b = oracle.spmv(A, np.ones(A.n_cols))
    st, x, stat = mg_solve(mats, f2c, b, fmt=fmt)
    assert st == 0 and stat["status"] == 0
    assert oracle.relres(A, b, x) <= 1e-10
    assert np.abs(x - 1).max() < 1e-7
    if A.n_rows <= 20000:
        colors = [gs.greedy_coloring(m) for m in mats]
        _, it_ref, _ = gs.pcg_mg(mats, f2c, colors, b)
        assert abs(stat["iters"] - it_ref) <= 1
        _, it_gs, _ = gs.pcg(A, b, colors[0])
        assert stat["iters"] < it_gs


@pytest.mark.parametrize("levels,k", [(3, 1), (3, 4), (4, 3), (1, 3), (2, 2)])
def test_mg_iterates_match_oracle(levels, k):
    """Stopped after k iterations, the iterate equals the oracle's k-th
    MG-preconditioned iterate element by element (non-uniform right-hand
    side; a 16 x 16 x 8 grid and its coarse levels, the coarsest 2 x 2 x 1)."""
    from oracle import gs

    say("case: mg iterates", levels, k)
    mats, f2c = stencil_hierarchy(16, 16, 8, levels)
    b = uniform_vector(mats[0].n_rows, seed=11) - 0.5
    st, x, stat = mg_solve(mats, f2c, b, max_iter=k)
    assert st == -7 and stat["iters"] == k
    colors = [gs.greedy_coloring(m) for m in mats]
    x_ref, it_ref, _ = gs.pcg_mg(mats, f2c, colors, b, max_iter=k)
    assert it_ref == k
    assert np.max(np.abs(x - x_ref)) <= 1e-11 * np.max(np.abs(x_ref))


def test_mg_rejects_bad_hierarchies():
    say("case: mg errors")
    mats, f2c = stencil_hierarchy(8, 8, 8, 3)
    b = np.ones(mats[0].n_rows)
    bad = [f.copy() for f in f2c]
    bad[1][3] = mats[1].n_rows  # out of range for level 1
    assert mg_solve(mats, bad, b)[0] == -1
    bad = [f.copy() for f in f2c]
    bad[0][5] = bad[0][4]  # repeated entry
    assert mg_solve(mats, bad, b)[0] == -1
    assert mg_solve([mats[0], mats[0]], [np.arange(mats[0].n_rows, dtype=np.int32)], b)[0] == 0  # identity map
    assert mg_solve([mats[1], mats[0]], [np.arange(mats[0].n_rows, dtype=np.int32)], b[:mats[1].n_rows])[0] == -1
    # a coarse level without its diagonal
    C = mats[2]
    rows = np.repeat(np.arange(C.n_rows), np.diff(C.row_ptr))
    keep = ~((rows == 1) & (C.col == 1))
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows[keep], minlength=C.n_rows))])
    Cb = CSR(C.n_rows, C.n_cols, rp, C.col[keep], C.val[keep])
    assert mg_solve([mats[0], mats[1], Cb], f2c, b)[0] == -1
    st, x, stat = mg_solve(mats, f2c, np.zeros_like(b))
    assert st == 0 and stat["iters"] == 0 and np.all(x == 0)
    st, x, stat = mg_solve(mats, f2c, oracle.spmv(mats[0], np.ones(mats[0].n_rows)))
    assert st == 0 and np.abs(x - 1).max() < 1e-7


def test_preconditioned_solves_of_an_empty_system():
    """n = 0: modes 0 and 2 and the one-level MG solve return at once with
    status OK and no iteration."""
    say("case: empty preconditioned")
    torch = torch_mod()
    P = lib()
    E = CSR(0, 0, np.zeros(1, dtype=np.int64), np.zeros(0, dtype=np.int32), np.zeros(0))
    M = compress(E)
    b = torch.zeros(0, dtype=torch.float64, device="cuda")
    for mode in (0, 2):
        st, _, stats = P.cg_solve(M, b, mode=mode)
        assert st == 0 and stats[0]["iters"] == 0
    st, x, stat = P.cg_solve_mg([M], [], b)
    assert st == 0 and stat["iters"] == 0 and x.numel() == 0


def test_mg_full_size_192():
    """The benchmark's MG solve: 192^3 and its 96/48/24 levels, DIT, b = A*1.
    Checked by properties: 1e-10 in the oracle's own residual, x = 1 to 1e-7,
    and fewer iterations than the single-sweep preconditioner (mode 2) on the
    same matrix, which in turn needs fewer than plain CG (302 on this grid)."""
    say("case: mg full size 192^3")
    mats, f2c = stencil_hierarchy(192, 192, 192, 4)
    A = mats[0]
    b = oracle.spmv(A, np.ones(A.n_cols))
    st, x, stat = mg_solve(mats, f2c, b)
    assert st == 0 and stat["status"] == 0
    assert oracle.relres(A, b, x) <= 1e-10
    assert np.abs(x - 1).max() < 1e-7
    st2, _, stats2 = solve(A, b, mode=2)
    assert st2 == 0 and stat["iters"] < stats2[0]["iters"] < 302


def test_mg_levels_in_different_formats():
    """Each level is its own handle: a DIT fine level over ELL and DITV coarse
    levels gives the iterate of the all-DIT hierarchy (the formats decode to
    the same entries; the sums may differ in rounding order)."""
    say("case: mg mixed formats")
    torch = torch_mod()
    P = lib()
    mats, f2c = stencil_hierarchy(16, 16, 16, 3)
    b = uniform_vector(mats[0].n_rows, seed=13) - 0.5
    F = [torch.from_numpy(np.ascontiguousarray(f, dtype=np.int32)).cuda() for f in f2c]
    bt = torch.from_numpy(b).cuda()
    xs = []
    for fmts in (("DIT", "DIT", "DIT"), ("DIT", "ELL", "DITV")):
        Ms = [compress(m, fmt=f) for m, f in zip(mats, fmts)]
        st, x, stat = P.cg_solve_mg(Ms, F, bt, max_iter=4)
        torch.cuda.synchronize()
        assert st == -7 and stat["iters"] == 4
        xs.append(x.cpu().numpy())
    assert np.max(np.abs(xs[0] - xs[1])) <= 1e-11 * np.max(np.abs(xs[0]))


@pytest.mark.parametrize("fmt", ["DIT", "ELL"])
def test_pcg_irregular_matches_oracle(fmt):
    """Mode 2 on the irregular stencil (escape rows and raw values: the
    generic sweep kernel): the oracle's iteration count within 2, 1e-10 in
    the oracle's residual, x = 1."""
    from oracle import gs

    say("case: pcg irregular", fmt)
    A = stencil27_irregular(14, 12, 10, seed=4)
    b = oracle.spmv(A, np.ones(A.n_cols))
    st, x, stats = solve(A, b, fmt=fmt, mode=2)
    assert st == 0 and stats[0]["status"] == 0
    assert oracle.relres(A, b, x) <= 1e-10
    assert np.abs(x - 1).max() < 1e-7
    _, it_ref, _ = gs.pcg(A, b, gs.greedy_coloring(A))
    assert abs(stats[0]["iters"] - it_ref) <= 2
