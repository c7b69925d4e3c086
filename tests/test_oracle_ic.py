"""Pins of the oracle's red-black incomplete-Cholesky preconditioner (CPU
only): the factor is IC(0) (L L^T equals A on A's sparsity pattern), its
application agrees with the closed form that the red-black structure gives
(red cells couple only to black cells), M is symmetric positive definite,
and IC-preconditioned CG reaches the direct solution in fewer iterations
than Jacobi-PCG."""
import numpy as np
import pytest

import oracle
from oracle import direct, ic as oic
from oracle import mg as omg
from paper_2604_01800_amd import inputs


@pytest.mark.parametrize("nx,ny,bx,by", [(7, 5, 1.6, 0.9), (12, 9, 2.2, 1.3), (2, 2, 0.0, 0.0), (6, 11, 1.0, 2.5)])
def test_factor_is_ic0(nx, ny, bx, by):
    g = inputs.make_grid(nx, ny, bx, by)
    P = oic.RedBlackIC(g)
    Mp = (P.L @ P.Lt).toarray()
    Ap = P.Ap.toarray()
    on = Ap != 0
    assert np.abs(Mp[on] - Ap[on]).max() <= 1e-13 * np.abs(Ap).max()
    # L is lower triangular with A's lower pattern
    L = P.L.toarray()
    assert np.all(np.triu(L, 1) == 0)
    assert np.all((L != 0) <= (np.tril(Ap) != 0))


@pytest.mark.parametrize("nx,ny,bx,by", [(7, 5, 1.6, 0.9), (10, 8, 2.0, 1.4)])
def test_application_matches_red_black_closed_form(nx, ny, bx, by):
    """With D the diagonal, w the face weights and S_b = D_b - sum over the
    red neighbours r of w_br^2 / D_r: t = r / D on red cells, then
    z_b = (r_b + sum_r w_br t_r) / S_b on black cells, then
    z_r = (r_r + sum_b w_rb z_b) / D_r on red cells."""
    g = inputs.make_grid(nx, ny, bx, by)
    A = omg.fine_operator(g).toarray()
    D = np.diag(A)
    rng = np.random.default_rng(3)
    r = rng.standard_normal(nx * ny)
    j, i = np.divmod(np.arange(nx * ny), nx)
    red = (i + j) % 2 == 0
    W = -A.copy()
    np.fill_diagonal(W, 0.0)
    S = D - (W[:, red] ** 2 / D[red]).sum(axis=1)
    t = np.where(red, r / D, 0.0)
    zb = (r + W @ t) / S
    z = np.where(red, 0.0, zb)
    z = np.where(red, (r + W @ z) / D, z)
    got = oic.RedBlackIC(g).apply(r.reshape(ny, nx)).reshape(-1)
    np.testing.assert_allclose(got, z, rtol=1e-12, atol=1e-14 * np.abs(z).max())


def test_m_is_spd_and_close_to_a():
    g = inputs.make_grid(9, 8, 1.8, 1.2)
    P = oic.RedBlackIC(g)
    M = P.M()
    assert np.abs(M - M.T).max() <= 1e-13 * np.abs(M).max()
    assert np.linalg.eigvalsh(M).min() > 0.0
    # M - A is the dropped fill: black-black couplings two cells apart only
    A = omg.fine_operator(g).toarray()
    E = M - A
    j, i = np.divmod(np.arange(72), 9)
    red = (i + j) % 2 == 0
    assert np.abs(E[red]).max() <= 1e-13 * np.abs(A).max()
    assert np.abs(np.diag(E)).max() <= 1e-13 * np.abs(A).max()


def test_icpcg_beats_jacobi_and_matches_direct_solve(orc):
    g = inputs.make_grid(48, 40, 2.0, 1.5)
    f = inputs.gaussian_bumps(g, 5).astype(np.float32)
    b, _ = orc.rhs(g, f)
    P = oic.RedBlackIC(g)
    x_ic, s_ic, _ = orc.pcg(g, b, precond=2, pc=P.apply, tol=1e-10, max_iter=5000)
    _, s_j, _ = orc.pcg(g, b, precond=1, tol=1e-10, max_iter=5000)
    assert s_ic.converged and s_j.converged
    assert s_ic.iters_total < 0.8 * s_j.iters_total, (s_ic.iters_total, s_j.iters_total)
    xd = direct.separable_solve(g, b)
    x_ic = orc.remove_mean(x_ic)
    assert np.linalg.norm(x_ic - xd) <= 1e-8 * np.linalg.norm(xd)
