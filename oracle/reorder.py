"""Reverse Cuthill-McKee reordering -- TEST INFRASTRUCTURE ONLY.

Only the test-suite may use this module.  It shares no code with the GPU
library.

The paper traces the gap between its measured and theoretical SpMV speed to
the irregular access of x through large column offsets, and names reordering
of the matrix and the vector as the remedy (Section V, after Table II).  The
standard reordering for that purpose is reverse Cuthill-McKee (Cuthill and
McKee 1969; George 1971): a breadth-first numbering that keeps each row's
neighbours close to it, reversed.

Definition used here (the rules the literature leaves open are fixed so the
result is unique):
  * the graph is the pattern of A + A^T without the diagonal; deg(v) is the
    number of distinct neighbours of v;
  * while unnumbered vertices remain, the next component starts at the
    unnumbered vertex of least (deg, index);
  * Cuthill-McKee: take the numbered vertices in order; each appends its
    unnumbered neighbours in order of (deg, index);
  * reverse Cuthill-McKee is that sequence reversed.
Returns perm with perm[k] = the old index of the vertex numbered k.

``permute`` forms B = P A P^T: row k of B is row perm[k] of A with every
column j renamed rank[j] (rank = inverse of perm), columns ascending.

Pins (tests/test_oracle_reorder.py): a path graph under any labelling comes
out as the path, bandwidth 1; a star comes out leaves-center-leaf in a closed
form; a hand-numbered two-component graph with degree ties; a second,
level-by-level formulation (each vertex of a level ordered by the least
number among its neighbours in the level before, then deg, index) agrees on
random graphs; ``permute`` keeps every entry, and B (P x) = P (A x).
"""
from __future__ import annotations

from collections import deque

import numpy as np


def neighbours(A) -> list:
    """Sorted distinct neighbours of every vertex in the pattern of A + A^T."""
    n = A.n_rows
    rp = np.asarray(A.row_ptr, dtype=np.int64)
    col = np.asarray(A.col, dtype=np.int64)
    nbr = [set() for _ in range(n)]
    for i in range(n):
        for k in range(int(rp[i]), int(rp[i + 1])):
            j = int(col[k])
            if j != i:
                nbr[i].add(j)
                nbr[j].add(i)
    return [sorted(s) for s in nbr]


def rcm(A) -> np.ndarray:
    """Reverse Cuthill-McKee permutation (perm[new] = old) of a square A."""
    if A.n_rows != A.n_cols:
        raise ValueError("reordering needs a square matrix")
    n = A.n_rows
    nbr = neighbours(A)
    deg = [len(s) for s in nbr]
    numbered = [False] * n
    order = []
    by_deg = sorted(range(n), key=lambda v: (deg[v], v))
    for s in by_deg:
        if numbered[s]:
            continue
        numbered[s] = True
        q = deque([s])
        while q:
            v = q.popleft()
            order.append(v)
            for u in sorted((u for u in nbr[v] if not numbered[u]), key=lambda u: (deg[u], u)):
                numbered[u] = True
                q.append(u)
    return np.array(order[::-1], dtype=np.int64)


def permute(A, perm):
    """B = P A P^T as CSR (row_ptr int64, col int32, val float64), columns ascending."""
    from synthetic import CSR

    perm = np.asarray(perm, dtype=np.int64)
    n = A.n_rows
    rank = np.empty(n, dtype=np.int64)
    rank[perm] = np.arange(n)
    rp = np.asarray(A.row_ptr, dtype=np.int64)
    lens = np.diff(rp)[perm]
    new_rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=new_rp[1:])
    col = np.empty(int(new_rp[-1]), dtype=np.int32)
    val = np.empty(int(new_rp[-1]), dtype=np.float64)
    for k in range(n):
        o = int(perm[k])
        c = rank[np.asarray(A.col[rp[o]:rp[o + 1]], dtype=np.int64)]
        v = np.asarray(A.val[rp[o]:rp[o + 1]], dtype=np.float64)
        s = np.argsort(c, kind="stable")
        col[new_rp[k]:new_rp[k + 1]] = c[s]
        val[new_rp[k]:new_rp[k + 1]] = v[s]
    return CSR(n, n, new_rp, col, val)


def bandwidth(A) -> int:
    """max |i - j| over the entries of A (0 for an empty or diagonal matrix)."""
    rows = np.repeat(np.arange(A.n_rows, dtype=np.int64), np.diff(A.row_ptr))
    if rows.size == 0:
        return 0
    return int(np.max(np.abs(rows - np.asarray(A.col, dtype=np.int64))))
