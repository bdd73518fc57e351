"""Seeded synthetic SDP instances with given block sizes, for the blocks the relaxations here do
not produce (the paper's 190 x 190 and 231 x 231 moment blocks).  Input construction only: no
arithmetic of the method.  Draws come from numpy's PCG64 generator seeded with `seed`.

The instance: m sparse rows, each with 1-6 random svec entries of one block (the last 8 rows
couple two blocks), standard-normal coefficients; b = A(X_f) for a random positive definite
X_f = G G^T / n + 0.1 I per block (so the instance is feasible); C = G G^T / n + I per block
(positive definite, so the objective is bounded below on the cone).  svec: column-major upper
triangle with sqrt(2) on the off-diagonal, the layout of the solver's problem arrays.
"""
from __future__ import annotations

import numpy as np


def _svec(M: np.ndarray) -> np.ndarray:
    i, j = np.triu_indices(M.shape[0])
    order = np.lexsort((i, j))  # by column, then row
    i, j = i[order], j[order]
    return M[i, j] * np.where(i == j, 1.0, np.sqrt(2.0))


def large_block_sdp(sizes, m: int, seed: int) -> dict:
    """Arrays of the instance: block_sizes (int32), boff (int64), nsvec, m, rowptr (int64),
    col (int32), val, b, C (float64)."""
    rng = np.random.default_rng(seed)
    sizes = np.array(sizes, np.int32)
    tri = sizes.astype(np.int64) * (sizes + 1) // 2
    boff = np.concatenate([[0], np.cumsum(tri)[:-1]]).astype(np.int64)
    nsvec = int(tri.sum())
    rows = []
    for r in range(m):
        ks = rng.choice(len(sizes), 2, replace=False) if r >= m - 8 else [rng.integers(len(sizes))]
        ent = {}
        for k in ks:
            for _ in range(rng.integers(1, 7)):
                ent[int(boff[k] + rng.integers(tri[k]))] = rng.standard_normal()
        rows.append(sorted(ent.items()))
    rowptr = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    col = np.array([c for r in rows for c, _ in r], np.int32)
    val = np.array([v for r in rows for _, v in r], np.float64)

    def pd(n, shift):
        G = rng.standard_normal((n, n))
        return G @ G.T / n + shift * np.eye(n)

    Xf = np.concatenate([_svec(pd(int(n), 0.1)) for n in sizes])
    C = np.concatenate([_svec(pd(int(n), 1.0)) for n in sizes])
    b = np.zeros(m)
    for r in range(m):
        a, e = rowptr[r], rowptr[r + 1]
        b[r] = float(np.dot(val[a:e], Xf[col[a:e]]))
    return dict(block_sizes=sizes, boff=boff, nsvec=nsvec, m=m, rowptr=rowptr, col=col, val=val, b=b, C=C)
