"""Pins of the oracle's reverse Cuthill-McKee reordering (oracle/reorder.py)."""
import numpy as np
import pytest

from oracle import reorder
from synthetic import CSR, stencil27, stencil27_irregular, uniform_vector


def graph(n, edges):
    """Symmetric CSR with unit diagonal from an undirected edge list."""
    rows = [i for i in range(n)] + [a for a, b in edges] + [b for a, b in edges]
    cols = [i for i in range(n)] + [b for a, b in edges] + [a for a, b in edges]
    order = np.lexsort((cols, rows))
    r, c = np.asarray(rows)[order], np.asarray(cols)[order]
    rp = np.concatenate([[0], np.cumsum(np.bincount(r, minlength=n))]).astype(np.int64)
    return CSR(n, n, rp, c.astype(np.int32), np.ones(len(c)))


def test_hand_numbered_two_components():
    """Worked by hand: component {0,3,5,6} (edges 0-3, 3-5, 3-6, 5-6) starts at
    0 (least degree, then index), numbers 3, then 5 and 6 (degree tie, index);
    component {1,2,4} (path 1-2-4) starts at 1.  CM = 0 3 5 6 1 2 4."""
    A = graph(7, [(0, 3), (3, 5), (3, 6), (5, 6), (1, 2), (2, 4)])
    assert reorder.rcm(A).tolist() == [4, 2, 1, 6, 5, 3, 0]


@pytest.mark.parametrize("center,n", [(2, 5), (0, 6), (5, 6)])
def test_star(center, n):
    """A star: CM starts at the least-index leaf, then the center, then the
    other leaves by index; RCM is that reversed."""
    leaves = [v for v in range(n) if v != center]
    A = graph(n, [(center, v) for v in leaves])
    cm = [leaves[0], center] + leaves[1:]
    assert reorder.rcm(A).tolist() == cm[::-1]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_path_under_any_labelling(seed):
    """A path whose vertices carry random labels comes out as the path, from
    the end with the larger label, and the reordered matrix has bandwidth 1."""
    n = 40
    p = np.random.default_rng(seed).permutation(n)
    A = graph(n, [(int(p[k]), int(p[k + 1])) for k in range(n - 1)])
    perm = reorder.rcm(A)
    path = p.tolist() if p[0] > p[-1] else p[::-1].tolist()
    assert perm.tolist() == path
    assert reorder.bandwidth(reorder.permute(A, perm)) == 1


def _rcm_by_levels(A):
    """The same numbering computed level by level: the vertices of the next
    level ordered by (least CM number among their neighbours in the level
    before, degree, index)."""
    nbr = reorder.neighbours(A)
    deg = [len(s) for s in nbr]
    n = A.n_rows
    num = [-1] * n
    order = []
    for s in sorted(range(n), key=lambda v: (deg[v], v)):
        if num[s] >= 0:
            continue
        num[s] = len(order)
        order.append(s)
        level = [s]
        while level:
            nxt = {}
            for v in level:
                for u in nbr[v]:
                    if num[u] < 0:
                        nxt[u] = min(nxt.get(u, n), num[v])
            level = sorted(nxt, key=lambda u: (nxt[u], deg[u], u))
            for u in level:
                num[u] = len(order)
                order.append(u)
    return order[::-1]


@pytest.mark.parametrize("seed", range(6))
def test_level_formulation_agrees(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 60))
    m = int(rng.integers(0, 3 * n))
    edges = {(int(a), int(b)) for a, b in rng.integers(0, n, size=(m, 2)) if a != b}
    A = graph(n, sorted(edges))
    assert reorder.rcm(A).tolist() == _rcm_by_levels(A)


def test_permute_keeps_the_operator():
    A = stencil27_irregular(7, 6, 5, seed=2)
    perm = np.random.default_rng(3).permutation(A.n_rows)
    B = reorder.permute(A, perm)
    x = uniform_vector(A.n_rows, seed=4)
    rows = lambda M: np.repeat(np.arange(M.n_rows), np.diff(M.row_ptr))
    Ax = np.bincount(rows(A), weights=A.val * x[A.col], minlength=A.n_rows)
    Bx = np.bincount(rows(B), weights=B.val * x[perm][B.col], minlength=B.n_rows)
    assert np.allclose(Bx, Ax[perm], rtol=0, atol=1e-12)
    assert B.nnz == A.nnz
    for k in range(B.n_rows):
        c = B.col[B.row_ptr[k]:B.row_ptr[k + 1]]
        assert np.all(np.diff(c) > 0)


def test_rcm_undoes_a_scrambled_stencil():
    """A 27-point stencil under a random labelling has bandwidth near n; after
    RCM the bandwidth is of the order of a grid plane."""
    A = stencil27(10, 9, 8)
    p = np.random.default_rng(5).permutation(A.n_rows)
    S = reorder.permute(A, p)
    assert reorder.bandwidth(S) > A.n_rows // 2
    R = reorder.permute(S, reorder.rcm(S))
    assert reorder.bandwidth(R) <= 4 * 10 * 9
