"""TEST INFRASTRUCTURE — FP64 reference of the multigrid preconditioner.

The paper's strongest CG-type solver is a 4-level multigrid-preconditioned CG
(MGPCG-4, Sec. 2.5): a V-cycle with a Chebyshev polynomial smoother, two pre-
and two post-smoothing iterations per level, and an exact solve on the
coarsest level. The paper builds its hierarchy by smoothed aggregation; on a
tensor-product grid this reference builds it geometrically, as stated here:

* Hierarchy: level l+1 merges each 2 x 2 block of cells of level l (nx and ny
  divisible by 2^(levels-1)). P_l is the piecewise-constant prolongation (a
  fine cell takes its parent's value); restriction is its transpose (the sum
  over the four children).
* Coarse operators: the Galerkin products A_{l+1} = P_l^T A_l P_l, formed
  literally as sparse matrix products.
* Smoother: the Chebyshev semi-iteration (Saad, Iterative Methods for Sparse
  Linear Systems, Sec. 12.3) on D^-1 A with D = diag(A_l), for the eigenvalue
  interval [lo * 2, 2]: 2 bounds the spectrum of D^-1 A for these operators
  (zero row sums, non-positive off-diagonals: Gershgorin), lo = 0.1. Degree
  2 (two updates) before and after the coarse correction, from a zero initial
  guess on the way down.
* Coarsest level: the minimum-norm solution A_c^+ b (dense pseudo-inverse).
* V-cycle for A_l x = b: x = S(0, b); r = b - A_l x; e = V_{l+1}(P_l^T r);
  x = x + P_l e; x = S(x, b). The preconditioner of PCG is M^-1 = V_0.

Plain numpy/scipy, single-threaded, no blocking or fusion; shares no code
with the GPU library.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

CHEB_HI = 2.0
CHEB_LO_FRAC = 0.1
CHEB_DEGREE = 2


def fine_operator(g) -> sp.csr_matrix:
    """The finite-volume operator of Eq. 10 on grid g as a sparse matrix
    (index j * nx + i): face weight (face length) / (centre distance) on
    interior faces, boundary faces dropped."""
    nx, ny = int(g.nx), int(g.ny)
    xc, yc, hx, hy = (np.asarray(a, np.float64) for a in (g.xc, g.yc, g.hx, g.hy))
    rows, cols, vals = [], [], []

    def face(c0, c1, w):
        rows.extend([c0, c1, c0, c1])
        cols.extend([c0, c1, c1, c0])
        vals.extend([w, w, -w, -w])

    for j in range(ny):
        for i in range(nx - 1):
            face(j * nx + i, j * nx + i + 1, hy[j] / (xc[i + 1] - xc[i]))
    for j in range(ny - 1):
        for i in range(nx):
            face(j * nx + i, (j + 1) * nx + i, hx[i] / (yc[j + 1] - yc[j]))
    return sp.csr_matrix((vals, (rows, cols)), shape=(nx * ny, nx * ny))


def prolongation(nx: int, ny: int) -> sp.csr_matrix:
    """Piecewise-constant prolongation from the (nx/2, ny/2) grid of merged
    2 x 2 blocks to the (nx, ny) grid."""
    rows = np.arange(nx * ny)
    j, i = np.divmod(rows, nx)
    cols = (j // 2) * (nx // 2) + i // 2
    return sp.csr_matrix((np.ones(nx * ny), (rows, cols)), shape=(nx * ny, (nx // 2) * (ny // 2)))


class Hierarchy:
    def __init__(self, g, levels: int = 4, lo_frac: float = CHEB_LO_FRAC, degree: int = CHEB_DEGREE):
        nx, ny = int(g.nx), int(g.ny)
        if levels < 1 or nx % (1 << (levels - 1)) or ny % (1 << (levels - 1)):
            raise ValueError("nx and ny must be divisible by 2^(levels-1)")
        self.levels, self.lo, self.degree = levels, lo_frac * CHEB_HI, degree
        self.A, self.P, self.shape = [fine_operator(g)], [], [(ny, nx)]
        for _ in range(levels - 1):
            P = prolongation(nx, ny)
            self.P.append(P)
            self.A.append((P.T @ self.A[-1] @ P).tocsr())
            nx, ny = nx // 2, ny // 2
            self.shape.append((ny, nx))
        self.D = [A.diagonal() for A in self.A]
        self.Ac_pinv = np.linalg.pinv(self.A[-1].toarray())

    def smooth(self, l: int, x: np.ndarray, b: np.ndarray) -> np.ndarray:
        """Chebyshev semi-iteration of the chosen degree on D^-1 A over
        [lo, 2], from x."""
        A, D = self.A[l], self.D[l]
        theta = 0.5 * (CHEB_HI + self.lo)
        delta = 0.5 * (CHEB_HI - self.lo)
        sigma = theta / delta
        rho = 1.0 / sigma
        r = b - A @ x
        d = r / D / theta
        for k in range(self.degree):
            x = x + d
            if k == self.degree - 1:
                break
            r = r - A @ d
            rho_next = 1.0 / (2.0 * sigma - rho)
            d = rho_next * rho * d + (2.0 * rho_next / delta) * (r / D)
            rho = rho_next
        return x

    def vcycle(self, b: np.ndarray, l: int = 0) -> np.ndarray:
        b = np.asarray(b, np.float64).reshape(-1)
        if l == self.levels - 1:
            return self.Ac_pinv @ b
        x = self.smooth(l, np.zeros_like(b), b)
        r = b - self.A[l] @ x
        e = self.vcycle(self.P[l].T @ r, l + 1)
        x = x + self.P[l] @ e
        return self.smooth(l, x, b)

    def apply(self, r: np.ndarray) -> np.ndarray:
        """z = M^-1 r for a field r [ny, nx]."""
        return self.vcycle(r).reshape(self.shape[0])

