"""Runs the library's kernels through the bounds-checked build
(libspmvc_check.so, loaded through SPMVC_LIBRARY) on every format and kernel
family and prints the violation count; each result is also checked against
the oracle.  Started as a separate process by test_gpu_checked_build.py
(the binding holds one library per process)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import oracle  # noqa: E402
import paper_1612_00530_amd as P  # noqa: E402
from oracle import gs  # noqa: E402
from synthetic import CSR, batched_grids, stencil27, stencil27_irregular, uniform_vector  # noqa: E402


def rel_err(A, x, y, yref):
    absA = CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, np.abs(A.val))
    s = oracle.spmv(absA, np.abs(x))
    d = np.abs(y - yref)
    return float((d[s > 0] / s[s > 0]).max()) if (s > 0).any() else float(d.max())


def main():
    assert P.LIB_PATH.endswith("libspmvc_check.so"), P.LIB_PATH
    P.load()
    n0, checked = P.check_violations()
    assert checked, "not the checked build"
    # the detector itself: an index out of range is reported once, then reset
    P.check_probe(2, 3)
    assert P.check_violations()[0] == 0
    P.check_probe(3, 3)
    assert P.check_violations()[0] == 1
    P.check_probe(-1, 3)
    assert P.check_violations()[0] == 1
    assert P.check_violations()[0] == 0
    print("probe ok", flush=True)
    dev = "cuda"
    mats = [stencil27(21, 18, 15), stencil27_irregular(20, 18, 15, seed=4), stencil27(40, 37, 23)]
    for A in mats:
        rp, col, val = (torch.from_numpy(a).to(dev) for a in (A.row_ptr, A.col, A.val))
        x = uniform_vector(A.n_cols, seed=1)
        xt = torch.from_numpy(x).to(dev)
        yref = oracle.spmv(A, x)
        for fmt in ("ELL", "DT", "DIT", "DITV", "BMASK"):
            M = P.compress(rp, col, val, n_cols=A.n_cols, fmt=fmt)
            for rows, lds in ((256, 1), (512, 1), (768, 1), (1024, 1), (512, 2), (512, 0)):
                M.set_config(rows, lds)
                y = M.spmv(xt).cpu().numpy()
                assert rel_err(A, x, y, yref) <= 1e-14, (fmt, rows, lds)
                M.spmv(xt.float())
            for mode in (3, 2, 1, 0):
                M.set_block_mode(mode)
                for nrhs in (2, 3, 8):
                    X = np.stack([uniform_vector(A.n_cols, seed=10 + r) for r in range(nrhs)], axis=1)
                    Y = M.spmv_block(torch.from_numpy(X).to(dev)).cpu().numpy()
                    Yref = oracle.spmv_block(A, X)
                    for r in range(nrhs):
                        assert rel_err(A, X[:, r], Y[:, r], Yref[:, r]) <= 1e-14, (fmt, mode, nrhs)
            b = oracle.spmv(A, np.ones(A.n_cols))
            for mode in (0, 1, 2, 3):
                st, xs, _ = P.cg_solve(M, torch.from_numpy(b).to(dev), mode=mode)
                assert st == 0 and oracle.relres(A, b, xs[0].cpu().numpy()) <= 1e-10, (fmt, mode)
            color = gs.greedy_coloring(A)
            xg = torch.zeros(A.n_rows, dtype=torch.float64, device=dev)
            M.symgs(torch.from_numpy(b).to(dev), xg)
            ref = gs.symgs(A, b, np.zeros(A.n_rows), color)
            assert np.abs(xg.cpu().numpy() - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max()), fmt
            st, xn, _ = P.cg_solve_noalloc(M, torch.from_numpy(b).to(dev))
            assert st == 0 and oracle.relres(A, b, xn.cpu().numpy()) <= 1e-10, fmt
            print("ok", fmt, A.n_rows, flush=True)
    # batched pairs (window-phased and lane-group SpMV forms)
    grids = batched_grids(5, 8, 20, seed=3)
    Ms, Bs, As = [], [], []
    for g in grids:
        A = stencil27(*g)
        As.append(A)
        rp, col, val = (torch.from_numpy(a).to(dev) for a in (A.row_ptr, A.col, A.val))
        Ms.append(P.compress(rp, col, val, n_cols=A.n_cols, fmt="DIT"))
        Bs.append(torch.from_numpy(np.stack([uniform_vector(A.n_rows, seed=r) for r in range(4)], 1)).to(dev))
    for form in ("0,8", "1,8", "2,32"):
        os.environ["SPMVC_BATCHED_SPMV"] = form
        st, xs, _ = P.cg_solve(Ms, Bs, nrhs=4)
        assert st == 0, form
        for A, Bt, Xt in zip(As, Bs, xs):
            for r in range(4):
                assert oracle.relres(A, Bt[:, r].cpu().numpy(), Xt[:, r].cpu().numpy()) <= 1e-10
    n, checked = P.check_violations()
    print(f"violations {n}", flush=True)
    return 0 if n == 0 else 1


if __name__ == "__main__":
    sys.exit(main())
