"""GPU reverse Cuthill-McKee (spmv_rcm) and symmetric permutation (spmv_permute)
against the oracle (oracle/reorder.py): permutations and permuted matrices
compared exactly, then the SpMV of the reordered matrix."""
import sys

import numpy as np
import pytest

import oracle
from oracle import reorder
from synthetic import CSR, stencil27, stencil27_irregular, uniform_vector

from gpu_util import compress, lib, max_rel_err, same_bits, to_dev, torch_mod

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def scrambled(A, seed):
    p = np.random.default_rng(seed).permutation(A.n_rows)
    return reorder.permute(A, p)


def graph(n, edges, diag=True):
    rows = ([i for i in range(n)] if diag else []) + [a for a, b in edges] + [b for a, b in edges]
    cols = ([i for i in range(n)] if diag else []) + [b for a, b in edges] + [a for a, b in edges]
    order = np.lexsort((cols, rows))
    r, c = np.asarray(rows, dtype=np.int64)[order], np.asarray(cols, dtype=np.int64)[order]
    rp = np.concatenate([[0], np.cumsum(np.bincount(r, minlength=n))]).astype(np.int64)
    return CSR(n, n, rp, c.astype(np.int32), np.arange(1, len(c) + 1, dtype=np.float64))


def gpu_rcm(A):
    torch = torch_mod()
    rp, col, _ = to_dev(A)
    perm = lib().rcm(rp, col)
    torch.cuda.synchronize()
    return perm.cpu().numpy().astype(np.int64)


def random_graph(seed, n):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(0, 2 * n))
    edges = sorted({(int(min(a, b)), int(max(a, b))) for a, b in rng.integers(0, n, size=(m, 2)) if a != b})
    return graph(n, edges, diag=bool(seed % 2))


CASES = {
    "stencil 16^3": lambda: stencil27(16, 16, 16),
    "scrambled stencil 10x9x8": lambda: scrambled(stencil27(10, 9, 8), 1),
    "scrambled irregular 13x11x7": lambda: scrambled(stencil27_irregular(13, 11, 7, seed=2), 3),
    "random graph 300 (components, isolated)": lambda: random_graph(4, 300),
    "random graph 1000 no diagonal": lambda: random_graph(5, 1000),
    "single vertex": lambda: graph(1, []),
    "path 2": lambda: graph(2, [(0, 1)]),
    "scrambled stencil 32^3": lambda: scrambled(stencil27(32, 32, 32), 6),
}


@pytest.mark.parametrize("name", list(CASES))
def test_rcm_matches_oracle(name):
    say("case: rcm", name)
    A = CASES[name]()
    assert np.array_equal(gpu_rcm(A), reorder.rcm(A))


@pytest.mark.parametrize("name", ["scrambled irregular 13x11x7", "random graph 300 (components, isolated)",
                                  "single vertex"])
def test_permute_matches_oracle(name):
    say("case: permute", name)
    torch = torch_mod()
    A = CASES[name]()
    perm = np.random.default_rng(7).permutation(A.n_rows).astype(np.int32)
    rp, col, val = to_dev(A)
    out = lib().permute(rp, col, val, torch.from_numpy(perm).cuda())
    torch.cuda.synchronize()
    B = reorder.permute(A, perm)
    assert np.array_equal(out[0].cpu().numpy(), B.row_ptr)
    assert np.array_equal(out[1].cpu().numpy(), B.col)
    assert same_bits(out[2].cpu().numpy(), B.val)


def test_empty_matrix():
    say("case: rcm empty")
    torch = torch_mod()
    P = lib()
    rp = torch.zeros(1, dtype=torch.int64, device="cuda")
    col = torch.zeros(0, dtype=torch.int32, device="cuda")
    assert P.rcm(rp, col).numel() == 0
    out = P.permute(rp, col, torch.zeros(0, dtype=torch.float64, device="cuda"), torch.zeros(0, dtype=torch.int32, device="cuda"))
    assert out[0].cpu().tolist() == [0]


def test_rejects_bad_inputs():
    say("case: reorder errors")
    torch = torch_mod()
    P = lib()
    asym = graph(4, [(0, 1)])
    keep = ~((np.repeat(np.arange(4), np.diff(asym.row_ptr)) == 1) & (asym.col == 0))
    rows = np.repeat(np.arange(4), np.diff(asym.row_ptr))[keep]
    A1 = CSR(4, 4, np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=4))]), asym.col[keep], asym.val[keep])
    with pytest.raises(P.SpmvcError) as e:
        gpu_rcm(A1)
    assert e.value.status == -1
    bad = CSR(3, 3, np.array([0, 2, 3, 4]), np.array([1, 0, 1, 2], dtype=np.int32), np.ones(4))
    with pytest.raises(P.SpmvcError) as e:
        gpu_rcm(bad)
    assert e.value.status == -3
    A = stencil27(3, 3, 2)
    rp, col, val = to_dev(A)
    p = torch.arange(A.n_rows, dtype=torch.int32, device="cuda")
    p[3] = 2
    with pytest.raises(P.SpmvcError) as e:
        P.permute(rp, col, val, p)
    assert e.value.status == -1
    p[3] = A.n_rows
    with pytest.raises(P.SpmvcError):
        P.permute(rp, col, val, p)
    assert np.array_equal(gpu_rcm(A), reorder.rcm(A))  # still usable


@pytest.mark.parametrize("fmt", ["AUTO", "DIT", "ELL"])
def test_spmv_after_reordering(fmt):
    """Scrambled 24^3 stencil -> RCM -> permute -> compress -> y = B x'; equals
    the oracle SpMV of the oracle-permuted matrix, and (A x)[perm]."""
    say("case: spmv after rcm", fmt)
    torch = torch_mod()
    P = lib()
    S = scrambled(stencil27(24, 24, 24), 8)
    rp, col, val = to_dev(S)
    perm = P.rcm(rp, col)
    brp, bcol, bval = P.permute(rp, col, val, perm)
    M = P.compress(brp, bcol, bval, n_cols=S.n_cols, fmt=fmt)
    x = uniform_vector(S.n_rows, seed=9)
    pn = perm.cpu().numpy().astype(np.int64)
    y = M.spmv(torch.from_numpy(x[pn]).cuda()).cpu().numpy()
    B = reorder.permute(S, pn)
    assert max_rel_err(B, x[pn], y, oracle.spmv(B, x[pn])) <= 1e-14
    assert max_rel_err(B, x[pn], y, oracle.spmv(S, x)[pn]) <= 1e-14
    # the start is a corner (least degree); the breadth-first levels are the
    # shells max(|di|, |dj|, |dk|) = L around it, the largest (L = 23) holding
    # 3 L^2 + 3 L + 1 = 1657 points, and a row's neighbours lie in its own
    # shell or the adjacent ones
    assert reorder.bandwidth(B) <= 2 * (3 * 23 ** 2 + 3 * 23 + 1)
    assert reorder.bandwidth(B) < reorder.bandwidth(S) // 5


def test_full_size_104_scrambled():
    """The benchmark's case: the 104^3 stencil under a random labelling (seed 0)
    applied with spmv_permute, then RCM.  Checked by properties that hold at
    any size: perm is a permutation; the reordered bandwidth is the largest
    breadth-first shell around the corner the numbering starts from,
    3 L^2 + 3 L + 1 with L = 103; the first row of the RCM order (the last
    numbered) is a corner's far shell and the last row is a corner; SpMV of
    the reordered matrix on sampled rows equals (A x)[perm] computed row by
    row from the natural stencil."""
    say("case: rcm full size 104^3")
    torch = torch_mod()
    P = lib()
    g = 104
    A = stencil27(g, g, g)
    rp, col, val = to_dev(A)
    scr = np.random.default_rng(0).permutation(A.n_rows).astype(np.int32)
    srp, scol, sval = P.permute(rp, col, val, torch.from_numpy(scr).cuda())
    perm = P.rcm(srp, scol)
    brp, bcol, bval = P.permute(srp, scol, sval, perm)
    torch.cuda.synchronize()
    pn = perm.cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(pn), np.arange(A.n_rows))
    rows = torch.repeat_interleave(torch.arange(A.n_rows, device="cuda"), brp[1:] - brp[:-1])
    assert int((rows - bcol.long()).abs().max().item()) == 3 * 103 ** 2 + 3 * 103 + 1
    # natural index of the vertex numbered k: scr maps scrambled -> natural
    nat = scr.astype(np.int64)[pn]
    ix, iy, iz = nat % g, (nat // g) % g, nat // (g * g)
    corner = lambda i: (i == 0) | (i == g - 1)
    assert corner(ix[-1]) and corner(iy[-1]) and corner(iz[-1])
    x = uniform_vector(A.n_rows, seed=3)
    M = P.compress(brp, bcol, bval, n_cols=A.n_cols, fmt="AUTO")
    xb = torch.from_numpy(x[nat]).cuda()
    y = M.spmv(xb).cpu().numpy()
    sample = np.random.default_rng(4).choice(A.n_rows, 4000, replace=False)
    for k in sample[:4000]:
        i = int(nat[k])
        lo, hi = int(A.row_ptr[i]), int(A.row_ptr[i + 1])
        ref = float(np.dot(A.val[lo:hi], x[A.col[lo:hi]]))
        scale = float(np.dot(np.abs(A.val[lo:hi]), np.abs(x[A.col[lo:hi]])))
        assert abs(y[k] - ref) <= 1e-14 * scale


def test_rows_beyond_the_length_limit_are_refused():
    """A row of more than 1024 entries (an arrowhead: vertex 0 coupled to all)
    is refused with SPMVC_EUNSUPPORTED by both calls before any ordering
    kernel runs; 1024 entries pass."""
    say("case: reorder row-length limit")
    torch = torch_mod()
    P = lib()
    for n, ok in ((1025, False), (1024, True)):
        A = graph(n, [(0, j) for j in range(1, n)])  # row 0: n entries with the diagonal
        if ok:
            assert np.array_equal(gpu_rcm(A), reorder.rcm(A))
            continue
        with pytest.raises(P.SpmvcError) as e:
            gpu_rcm(A)
        assert e.value.status == -8
        rp, col, val = to_dev(A)
        with pytest.raises(P.SpmvcError) as e:
            P.permute(rp, col, val, torch.arange(n, dtype=torch.int32, device="cuda"))
        assert e.value.status == -8
