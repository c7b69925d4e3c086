"""TEST INFRASTRUCTURE — direct solves of the pressure Poisson system.

Two routes to the minimum-norm solution x* = A^+ b that do not iterate:

* ``separable_solve``: the tensor-product method of Lynch, Rice & Thomas (1964).
  On a tensor grid the finite-volume operator of Eq. 10 splits as
      A = kron(Hy, Tx) + kron(Ty, Hx)
  (row-major index j*nx + i), where Hx = diag(hx) and Tx is the 1D Neumann
  operator (Tx u)_i = sum_nb (u_i - u_nb) / (xc_nb - xc_i) signed so Tx >= 0.
  The generalised eigenproblem Tx phi = mu Hx phi is solved through the
  symmetric tridiagonal Hx^-1/2 Tx Hx^-1/2, which decouples the 2D system into
  one tridiagonal solve (Ty + mu_k Hy) c_k = beta_k per x-mode. The mu = 0 mode
  is singular (constant null space) and is solved in the least-squares sense;
  the plain mean of the result is removed at the end, which gives A^+ b.
* ``dense_pinv_solve``: numpy's pseudo-inverse of the dense matrix (tiny grids).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import eigh_tridiagonal, solve_banded


def neumann_1d(xc: np.ndarray) -> np.ndarray:
    """Dense 1D operator T with (T u)_i = sum over neighbours (u_i - u_nb)/|dx|."""
    n = len(xc)
    w = 1.0 / np.diff(xc)
    T = np.zeros((n, n))
    for k in range(n - 1):
        T[k, k] += w[k]
        T[k + 1, k + 1] += w[k]
        T[k, k + 1] -= w[k]
        T[k + 1, k] -= w[k]
    return T


def kron_matrix(g) -> np.ndarray:
    """Dense A = kron(Hy, Tx) + kron(Ty, Hx) (for small grids only)."""
    Tx, Ty = neumann_1d(g.xc), neumann_1d(g.yc)
    return np.kron(np.diag(g.hy), Tx) + np.kron(Ty, np.diag(g.hx))


def dense_pinv_solve(g, b: np.ndarray) -> np.ndarray:
    A = kron_matrix(g)
    return (np.linalg.pinv(A, rcond=1e-12) @ b.reshape(-1)).reshape(g.ny, g.nx)


def separable_solve(g, b: np.ndarray) -> np.ndarray:
    """Minimum-norm solution of A x = b for b with zero sum, [ny, nx] FP64."""
    b = np.asarray(b, dtype=np.float64).reshape(g.ny, g.nx)
    wx = 1.0 / np.diff(g.xc)
    wy = 1.0 / np.diff(g.yc)
    # Tx diagonal / off-diagonal, then the symmetric scaling by Hx^-1/2.
    dx = np.zeros(g.nx)
    dx[:-1] += wx
    dx[1:] += wx
    s = 1.0 / np.sqrt(g.hx)
    mu, Q = eigh_tridiagonal(dx * s * s, -wx * s[:-1] * s[1:])
    Phi = s[:, None] * Q  # Phi^T Hx Phi = I, Phi^T Tx Phi = diag(mu)
    beta = b @ Phi  # [ny, nx-modes]
    dy = np.zeros(g.ny)
    dy[:-1] += wy
    dy[1:] += wy
    C = np.empty_like(beta)
    k0 = int(np.argmin(np.abs(mu)))
    for k in range(g.nx):
        if k == k0:
            Ty = np.diag(dy) - np.diag(wy, 1) - np.diag(wy, -1)
            C[:, k] = np.linalg.lstsq(Ty, beta[:, k], rcond=None)[0]
            continue
        ab = np.zeros((3, g.ny))
        ab[0, 1:] = -wy
        ab[1, :] = dy + mu[k] * g.hy
        ab[2, :-1] = -wy
        C[:, k] = solve_banded((1, 1), ab, beta[:, k])
    x = C @ Phi.T
    return x - x.mean()
