"""Pins of the Lanczos-Ritz reference (Sec. 2.3, Eqs. 14-16) against the dense
operator and the definition:

* V_m is orthonormal and orthogonal to the constant null vector, and
  V_m M V_m^T is the tridiagonal (alpha, beta) of the recurrence (Eq. 14),
  with M the dense finite-volume matrix built independently of the oracle's
  apply;
* a full run (m = N - 1, the whole range of M) gives as Ritz values exactly
  the nonzero eigenvalues of the dense matrix, and Ritz pairs with small
  residuals;
* the training vectors have unit norm and zero mean, and their energy on
  the Ritz vectors j <= b m is 81 times that on the others on average
  (Eq. 16), which a wrong weighting, index or ordering would break;
* the normal draws have zero mean and unit variance."""
import numpy as np
import pytest

import oracle
from oracle import direct, ritz
from paper_2604_01800_amd import inputs


def small_system(nx=7, ny=5, seed=0):
    g = inputs.make_grid(nx, ny, 1.6, 0.9)
    A = direct.kron_matrix(g)
    rng = np.random.default_rng(seed)
    return g, A, rng.standard_normal(nx * ny)


def test_lanczos_basis_and_tridiagonal():
    g, A, v0 = small_system()
    m = 12
    V, alpha, beta = ritz.lanczos(lambda x: oracle.apply(g, x.reshape(g.ny, g.nx)).ravel(), v0, m)
    assert V.shape == (m, g.nx * g.ny)
    np.testing.assert_allclose(V @ V.T, np.eye(m), atol=1e-12)
    assert np.abs(V.sum(axis=1)).max() <= 1e-12
    T = V @ A @ V.T
    want = np.diag(alpha) + np.diag(beta, 1) + np.diag(beta, -1)
    np.testing.assert_allclose(T, want, atol=1e-10 * np.abs(alpha).max())


def test_full_run_gives_the_spectrum():
    g, A, v0 = small_system(6, 5, seed=1)
    N = g.nx * g.ny
    V, alpha, beta = ritz.lanczos(lambda x: A @ x, v0, N - 1)
    theta, U = ritz.ritz(V, alpha, beta)
    lam = np.linalg.eigvalsh(A)
    np.testing.assert_allclose(theta, lam[1:], rtol=1e-10, atol=1e-10 * lam[-1])
    Q = V.T @ U
    res = np.linalg.norm(A @ Q - Q * theta, axis=0)
    assert res.max() <= 1e-9 * lam[-1]


def test_coefficients_are_standard_normal_with_weighting():
    m, b = 400, 0.6
    c = ritz.coefficients(m, 64, b, seed=5, step=3)
    jmax = int(np.floor(b * m))
    lo, hi = c[:, :jmax + 1] / 9.0, c[:, jmax + 1:]
    for x in (lo, hi):
        assert abs(x.mean()) <= 4 / np.sqrt(x.size)
        assert abs(x.var() - 1.0) <= 6 * np.sqrt(2.0 / x.size)
    # distinct steps and samples give distinct draws
    assert not np.allclose(c[0], c[1])
    assert not np.allclose(c[0], ritz.coefficients(m, 1, b, seed=5, step=4)[0])


def test_training_vectors_weight_the_low_spectrum():
    g, A, v0 = small_system(10, 8, seed=2)
    N = g.nx * g.ny
    m = N - 1
    V, alpha, beta = ritz.lanczos(lambda x: A @ x, v0, m)
    theta, U = ritz.ritz(V, alpha, beta)
    b = 0.6
    c = ritz.coefficients(m, 400, b, seed=9, step=0)
    R = ritz.training_vectors(V, U, c)
    np.testing.assert_allclose(np.linalg.norm(R, axis=1), 1.0, rtol=1e-12)
    assert np.abs(R.sum(axis=1)).max() <= 1e-12
    Q = V.T @ U
    P = (R @ Q) ** 2  # energy on each Ritz vector
    jmax = int(np.floor(b * m))
    ratio = P[:, :jmax + 1].mean() / P[:, jmax + 1:].mean()
    assert 81 * 0.8 <= ratio <= 81 * 1.25, ratio
    # and the weighted end is the low end of the spectrum: the mean Rayleigh
    # quotient is the 81:1 weighted mean of the Ritz values, below the plain mean
    rq = (R @ (A @ R.T)).diagonal().mean()
    w2 = np.where(np.arange(m) <= jmax, 81.0, 1.0)
    want = (w2 * theta).sum() / w2.sum()
    assert abs(rq / want - 1.0) <= 0.2, (rq, want)
    assert want < 0.8 * theta.mean()


@pytest.mark.parametrize("m", [1, 5])
def test_short_runs(m):
    g, A, v0 = small_system(5, 4, seed=3)
    V, alpha, beta = ritz.lanczos(lambda x: A @ x, v0, m)
    assert V.shape[0] == m and alpha.size == m and beta.size == m - 1
    theta, U = ritz.ritz(V, alpha, beta)
    lam = np.linalg.eigvalsh(A)
    assert lam[1] - 1e-9 <= theta.min() and theta.max() <= lam[-1] + 1e-9
