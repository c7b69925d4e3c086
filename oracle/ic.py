"""TEST INFRASTRUCTURE — FP64 reference of the incomplete-Cholesky
preconditioner in red-black ordering.

The paper's main comparison solver is incomplete-Cholesky PCG (ICPCG,
Sec. 2.5). Its triangular solves in the natural ordering run cell by cell
along the grid; in the red-black (checkerboard) ordering of the 5-point
operator, red cells couple only to black cells, so both triangular solves
become two passes over independent cells. This reference builds it as
stated here:

* Ordering: cell (i, j) is red when i + j is even; all red cells first, then
  all black cells, each in the natural order.
* Factor: IC(0) of the permuted operator, the textbook algorithm (Saad,
  Iterative Methods for Sparse Linear Systems, Sec. 10.3): row by row,
  L[k][k] = sqrt(a_kk - sum_{j<k} L[k][j]^2) and, for every (i, k) with i > k
  in the sparsity pattern of A, L[i][k] = (a_ik - sum_{j<k} L[i][j] L[k][j])
  / L[k][k]; entries outside A's pattern are dropped. M = L L^T.
* Application: z = M^-1 r by a forward substitution with L and a backward
  substitution with L^T (scipy's sparse triangular solve).

Plain numpy/scipy on small grids, no blocking or fusion; shares no code
with the GPU library (the sparse operator comes from oracle.mg).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mg import fine_operator


def red_black_order(nx: int, ny: int) -> np.ndarray:
    """Cell indices (j * nx + i) with every red cell (i + j even) before
    every black one, each colour in the natural order."""
    j, i = np.divmod(np.arange(nx * ny), nx)
    red = (i + j) % 2 == 0
    return np.concatenate([np.nonzero(red)[0], np.nonzero(~red)[0]])


def ic0(A: sp.csr_matrix) -> sp.csr_matrix:
    """IC(0) factor L (lower triangular, CSR) of the SPD-on-its-pattern
    matrix A, dropping every entry outside A's lower pattern."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    # rows below the diagonal in each column of A's lower pattern
    below = sp.tril(A, k=-1, format="csc")
    col_rows = [below.indices[below.indptr[k]:below.indptr[k + 1]] for k in range(n)]
    rows = [dict() for _ in range(n)]  # rows[i][j] = L[i][j], j <= i
    Ad = A.todok()
    for k in range(n):
        # the entries of row k left of the diagonal are final (columns < k)
        s = Ad.get((k, k), 0.0) - sum(v * v for j, v in rows[k].items() if j < k)
        if s <= 0.0:
            raise ValueError(f"IC(0) breaks down at row {k}")
        lkk = np.sqrt(s)
        rows[k][k] = lkk
        for i in col_rows[k]:
            t = Ad.get((i, k), 0.0) - sum(v * rows[k][j] for j, v in rows[i].items() if j < k and j in rows[k])
            rows[i][k] = t / lkk
    data, ri, ci = [], [], []
    for i, r in enumerate(rows):
        for j, v in r.items():
            ri.append(i)
            ci.append(j)
            data.append(v)
    return sp.csr_matrix((data, (ri, ci)), shape=(n, n))


class RedBlackIC:
    """M = L L^T from IC(0) of the red-black permuted operator of grid g."""

    def __init__(self, g):
        self.nx, self.ny = int(g.nx), int(g.ny)
        A = fine_operator(g)
        self.perm = red_black_order(self.nx, self.ny)
        self.Ap = A[self.perm][:, self.perm].tocsr()
        self.L = ic0(self.Ap)
        self.Lt = self.L.T.tocsr()

    def M(self) -> np.ndarray:
        """M in the natural ordering (dense; small grids)."""
        Mp = (self.L @ self.Lt).toarray()
        n = self.nx * self.ny
        out = np.empty((n, n))
        out[np.ix_(self.perm, self.perm)] = Mp
        return out

    def apply(self, r: np.ndarray) -> np.ndarray:
        """z = M^-1 r for a field r [ny, nx]."""
        rp = np.asarray(r, np.float64).reshape(-1)[self.perm]
        y = spla.spsolve_triangular(self.L, rp, lower=True)
        zp = spla.spsolve_triangular(self.Lt, y, lower=False)
        z = np.empty_like(zp)
        z[self.perm] = zp
        return z.reshape(self.ny, self.nx)
