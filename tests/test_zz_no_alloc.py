"""The allocation-free CG entry point (cg_solve_noalloc) against cg_solve.

Both run the same FP64 CG kernels; the no-allocation form keeps every buffer
in the library's static device region.  Two calls in a row (the second on a
smaller system in another format, so the region holds the first call's
contents) must each give cg_solve's result bit for bit and the oracle's
1e-10, without a single device allocation through the library's allocator
hook; a system beyond the region's limit is rejected.
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from synthetic import CSR, stencil27, uniform_vector

from gpu_util import compress, lib, same_bits, torch_mod

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_noalloc_equals_cg_solve_twice():
    torch = torch_mod()
    P = lib()
    L = P.load()
    count = {"alloc": 0}

    def _alloc(nbytes, stream, ctx):
        count["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(int(nbytes))

    def _free(ptr, stream, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    cases = [(stencil27(64, 60, 56), None, "DIT"),
             (stencil27(20, 18, 16), uniform_vector(20 * 18 * 16, seed=7), "ELL")]
    for A, b, fmt in cases:
        say("case: noalloc", fmt, A.n_rows)
        if b is None:
            b = oracle.spmv(A, np.ones(A.n_cols))
        M = compress(A, fmt=fmt)
        bt = torch.from_numpy(b).cuda()
        st_ref, xs, stats_ref = P.cg_solve(M, bt)
        torch.cuda.synchronize()
        x_ref = xs[0].cpu().numpy()
        x = torch.full_like(bt, 3.0)
        hooks = (P._ALLOC_FN(_alloc), P._FREE_FN(_free))
        assert L.spmvc_set_allocator(hooks[0], hooks[1], None) == 0
        try:
            st, x, stats = P.cg_solve_noalloc(M, bt, x)
            torch.cuda.synchronize()
        finally:
            assert L.spmvc_set_allocator(P._ALLOC_FN(), P._FREE_FN(), None) == 0
        assert count["alloc"] == 0
        xh = x.cpu().numpy()
        assert st == 0 and st_ref == 0 and stats["status"] == 0
        assert stats["iters"] == stats_ref[0]["iters"]
        assert same_bits(xh, x_ref)
        assert stats["relres_true"] == stats_ref[0]["relres_true"]
        assert oracle.relres(A, b, xh) <= 1e-10


def test_noalloc_rejects_systems_beyond_the_region():
    torch = torch_mod()
    P = lib()
    L = P.load()
    n = (1 << 21) + 1
    dev = "cuda"
    M = P.compress(torch.arange(n + 1, dtype=torch.int64, device=dev),
                   torch.arange(n, dtype=torch.int32, device=dev),
                   torch.full((n,), 2.0, dtype=torch.float64, device=dev), n_cols=n)
    b = torch.ones(n, dtype=torch.float64, device=dev)
    st, _, _ = P.cg_solve_noalloc(M, b)
    assert st == -1
    assert b"scratch limit" in L.spmvc_last_error()
    small = CSR(4, 4, np.arange(5), np.arange(4, dtype=np.int32), np.full(4, 2.0))
    Ms = compress(small)
    bs = torch.ones(4, dtype=torch.float64, device=dev)
    st, x, stats = P.cg_solve_noalloc(Ms, bs, max_iter=10, check_every=1)
    torch.cuda.synchronize()
    assert st == 0 and np.array_equal(x.cpu().numpy(), np.full(4, 0.5))
    x = torch.empty(4, dtype=torch.float64, device=dev)
    o = P.CgOpts(1e-10, 100, 1, 1e-5, 20, 16, 0)  # mixed mode is not offered here
    stat = (P.CgStat * 1)()
    assert L.cg_solve_noalloc(Ms.handle, ctypes.c_void_p(bs.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                              ctypes.byref(o), stat, None) == -1
