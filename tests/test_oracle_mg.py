"""Pins of the multigrid oracle (CPU only): the Galerkin coarse operators
against their closed tensor form, the Chebyshev smoother against its error
polynomial on generalized eigenvectors, the V-cycle's symmetry and
definiteness (what PCG needs of a preconditioner), its measured contraction
factor, the exact coarsest solve, and MG-PCG against the direct solve."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from paper_2604_01800_amd import inputs
from oracle import direct
from oracle import mg


def tensor_operator(hx, gx, hy, gy):
    """Operator of 1D arrays: widths h and face factors g (faces 0..n, zero at
    the walls): A = diag(hy) (x) T(gx) + T(gy) (x) diag(hx), index j * nx + i."""
    def T(g):
        return sp.diags([g[:-1] + g[1:], -g[1:-1], -g[1:-1]], [0, 1, -1])
    return (sp.kron(sp.diags(hy), T(gx)) + sp.kron(T(gy), sp.diags(hx))).tocsr()


def face_factors(c):
    g = np.zeros(len(c) + 1)
    g[1:-1] = 1.0 / np.diff(c)
    return g


def test_fine_operator_matches_oracle_apply(orc):
    g = inputs.make_grid(12, 10, 1.7, 0.6)
    A = mg.fine_operator(g)
    x = np.random.default_rng(0).standard_normal((10, 12))
    np.testing.assert_allclose(A @ x.reshape(-1), orc.apply(g, x).reshape(-1), atol=1e-12)


def test_galerkin_coarse_operator_closed_form():
    """P^T A P for the piecewise-constant prolongation is again the tensor
    five-point operator: merged widths, and at each surviving face the fine
    face's factor 1/(fine centre distance) (the internal faces of a 2 x 2
    block carry no flux of a blockwise-constant field)."""
    g = inputs.make_grid(16, 8, 2.1, 1.3)
    H = mg.Hierarchy(g, levels=3)
    hx, hy = np.asarray(g.hx), np.asarray(g.hy)
    gx, gy = face_factors(g.xc), face_factors(g.yc)
    for l in range(1, 3):
        hx, gx = hx[0::2] + hx[1::2], gx[0::2]
        hy, gy = hy[0::2] + hy[1::2], gy[0::2]
        want = tensor_operator(hx, gx, hy, gy)
        np.testing.assert_allclose(H.A[l].toarray(), want.toarray(), rtol=0, atol=1e-12 * abs(want).max())


def test_chebyshev_smoother_error_polynomial():
    """From x0 with b = 0 the smoother maps a generalized eigenvector v of
    (A, D) with eigenvalue lam to p(lam) v, p(t) = T_2((theta - t)/delta) /
    T_2(theta/delta), the degree-2 Chebyshev polynomial of the interval."""
    g = inputs.make_grid(8, 6, 1.5, 0.8)
    H = mg.Hierarchy(g, levels=1)
    A, D = H.A[0].toarray(), H.D[0]
    lam, V = sla.eigh(A, np.diag(D))
    assert lam.max() <= 2.0 + 1e-12  # the interval's upper end bounds the spectrum
    theta, delta = 0.5 * (2.0 + H.lo), 0.5 * (2.0 - H.lo)
    T2 = lambda t: 2 * t * t - 1
    for k in range(len(lam)):
        v = V[:, k]
        out = H.smooth(0, v.copy(), np.zeros_like(v))
        np.testing.assert_allclose(out, T2((theta - lam[k]) / delta) / T2(theta / delta) * v, atol=1e-12)


@pytest.mark.parametrize("levels", [2, 3])
def test_vcycle_is_symmetric_and_positive(levels):
    g = inputs.make_grid(32, 24, 1.8, 1.2)
    H = mg.Hierarchy(g, levels=levels)
    rng = np.random.default_rng(1)
    for _ in range(4):
        u = rng.standard_normal((24, 32))
        v = rng.standard_normal((24, 32))
        u -= u.mean()
        v -= v.mean()
        Mu, Mv = H.apply(u), H.apply(v)
        assert abs(np.sum(u * Mv) - np.sum(v * Mu)) <= 1e-12 * np.linalg.norm(u) * np.linalg.norm(Mv)
        assert np.sum(u * Mu) > 0


def _contraction(n, beta, levels, steps=40):
    g = inputs.make_grid(n, n, beta)
    H = mg.Hierarchy(g, levels=levels)
    A = H.A[0]
    e = np.random.default_rng(2).standard_normal(n * n)
    e -= e.mean()
    anorm = lambda v: np.sqrt(v @ (A @ v))
    factor = 0.0
    for _ in range(steps):
        e1 = e - H.vcycle(A @ e)
        e1 -= e1.mean()
        factor = anorm(e1) / anorm(e)
        e = e1 / anorm(e1)
    return factor


def test_vcycle_contraction_factor():
    """The V-cycle as a stationary iteration, e <- (I - M A) e, contracts the
    A-norm of the error (power iteration on zero-mean errors). On a uniform
    grid the two-grid factor of piecewise-constant aggregation does not grow
    with the grid (about 0.61 at 64^2 and 128^2); on stretched grids and with
    more levels it is larger but below 1, and CG accelerates it."""
    u64, u128 = _contraction(64, 0.0, 2), _contraction(128, 0.0, 2)
    assert u64 < 0.7 and abs(u128 - u64) < 0.02, (u64, u128)
    for n, beta, levels in [(48, 1.5, 2), (64, 1.75, 4)]:
        f = _contraction(n, beta, levels)
        assert 0.05 < f < 0.95, (n, levels, f)


def test_single_level_is_the_pseudo_inverse(orc):
    """With one level the preconditioner is the exact min-norm solve, and
    PCG converges in one iteration."""
    g = inputs.make_grid(12, 10, 1.6)
    H = mg.Hierarchy(g, levels=1)
    b, _ = orc.rhs(g, inputs.gaussian_bumps(g, 1))
    z = H.apply(b)
    assert abs(z.mean()) <= 1e-13 * np.abs(z).max()
    np.testing.assert_allclose(orc.apply(g, z), b, atol=1e-11 * np.abs(b).max())
    x, st, _ = orc.pcg(g, b, precond=2, pc=H.apply, tol=1e-10, max_iter=10)
    assert st.converged and st.iters_total == 1


def test_mgpcg_matches_direct_solve(orc):
    g = inputs.with_ellipse(inputs.make_grid(64, 48, 1.75, 2.2), np.random.default_rng(3))
    b, _ = orc.rhs(g, inputs.grf(g, 4))
    H = mg.Hierarchy(g, levels=4)
    x, st, _ = orc.pcg(g, b, precond=2, pc=H.apply, tol=1e-12, max_iter=500)
    xj, sj, _ = orc.pcg(g, b, precond=1, tol=1e-12, max_iter=20000)
    assert st.converged and sj.converged
    assert st.iters_total * 5 < sj.iters_total, (st.iters_total, sj.iters_total)
    xd = direct.separable_solve(g, b)
    x = orc.remove_mean(x)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)


def test_mg_hybrid_with_exact_direction_and_rejections(orc):
    """DLSM over MGPCG (Sec. 2.2 with the MG CG-type): with the exact error as
    the direction one line-search step solves the system; with rejected
    directions the hybrid still converges (restarted MG-PCG)."""
    g = inputs.make_grid(32, 32, 1.5)
    b, _ = orc.rhs(g, inputs.gaussian_bumps(g, 2))
    H = mg.Hierarchy(g, levels=3)
    Ap = np.linalg.pinv(mg.fine_operator(g).toarray())
    exact = lambda r: (Ap @ r.reshape(-1)).reshape(r.shape)
    x, st, _ = orc.hybrid(g, b, exact, precond=2, pc=H.apply, tol=1e-10, num_cg=1, num_dlsm=1, max_iter=10)
    assert st.converged and st.iters_total == 2 and st.iters_dlsm == 1
    x, st, _ = orc.hybrid(g, b, lambda r: np.zeros_like(r), precond=2, pc=H.apply, tol=1e-8, max_iter=400)
    assert st.converged and st.dlsm_rejected > 0
