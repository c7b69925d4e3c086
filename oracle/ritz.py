"""TEST INFRASTRUCTURE — reference of the Lanczos-Ritz training vectors.

Plain numpy/scipy, FP64; nothing here is shared with the GPU library, which
implements the same definition in its own kernels.

Definition (Sec. 2.3, Eqs. 14-16):
  * Lanczos on the operator M of Eq. 10 (here the finite-volume operator A,
    symmetric with the constant vector as null space): from a start vector
    v0, projected onto zero mean and normalised, m steps give an orthonormal
    V_m (rows v_0 .. v_{m-1}) and the tridiagonal T_m = V_m^T M V_m (Eq. 14)
    with diagonal alpha and off-diagonal beta. Every step orthogonalises the
    new vector against the normalised constant vector and all earlier
    Lanczos vectors, twice (classical Gram-Schmidt applied twice); the paper
    does not say how orthogonality is kept, and without this the Ritz
    vectors of a long run repeat.
  * Ritz pairs: T_m = U diag(theta) U^T with theta ascending, Q_m = V_m U;
    each eigenvector is signed so that its first component (along v_0) is
    not negative (the paper leaves the signs open; they change R^i).
  * Training vector i (Eqs. 15-16): R^i = Q c^i / |Q c^i|_2 with
    c^i_j = 9 N(0,1) for 0 <= j <= b m and N(0,1) otherwise (j counts from
    the lowest Ritz value, so the low end of the spectrum is weighted up).
  * The normal draws: Philox4x32-10 as in the right-hand-side generator
    (key = seed, counter = (j, s + 2^31, step mod 2^32, step div 2^32)), and
    c = sqrt(-2 ln u_0) cos(2 pi u_1) (Box-Muller). Setting bit 31 of the
    sample word keeps these draws apart from the generator's own.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import eigh_tridiagonal

from .datagen import philox_vec, to_unit


def lanczos(apply, v0, m):
    """m Lanczos steps (Eq. 14) with full re-orthogonalisation.

    apply(x) -> A x for x of shape [N] (FP64). Returns (V [m, N], alpha [m],
    beta [m - 1]); stops early, with fewer rows, if the Krylov space is
    exhausted (beta below 1e-12 of the largest alpha)."""
    v0 = np.asarray(v0, dtype=np.float64).ravel()
    N = v0.size
    e = np.full(N, 1.0 / np.sqrt(N))
    v = v0 - e * (e @ v0)
    V = [v / np.linalg.norm(v)]
    alpha, beta = [], []
    for j in range(m):
        w = apply(V[j])
        alpha.append(V[j] @ w)
        B = np.vstack([e[None]] + V)
        for _ in range(2):
            w = w - B.T @ (B @ w)
        if j + 1 == m:
            break
        b = np.linalg.norm(w)
        if b <= 1e-12 * max(abs(a) for a in alpha):
            break
        beta.append(b)
        V.append(w / b)
    return np.array(V), np.array(alpha), np.array(beta)


def ritz(V, alpha, beta):
    """Ritz values (ascending) and the eigenvectors U of T_m, signed so that
    U[0, j] >= 0."""
    theta, U = eigh_tridiagonal(alpha, beta)
    U = U * np.where(U[0] < 0.0, -1.0, 1.0)
    return theta, U


def coefficients(m, nb, b, seed, step):
    """c [nb, m] of Eq. 16 for samples 0 .. nb - 1."""
    c = np.empty((nb, m))
    jmax = int(np.floor(b * m))
    for s in range(nb):
        u = to_unit(philox_vec(np.arange(m), s + (1 << 31), step, seed))
        c[s] = np.sqrt(-2.0 * np.log(u[:, 0])) * np.cos(2.0 * np.pi * u[:, 1])
        c[s, :jmax + 1] *= 9.0
    return c


def training_vectors(V, U, c):
    """R [nb, N] of Eq. 15: R = Q c / |Q c| with Q = V^T U (columns q_j)."""
    Q = V.T @ U
    R = c @ Q.T
    return R / np.linalg.norm(R, axis=1, keepdims=True)
