"""Pins of the oracle's Jacobi-PCG and hybrid CG / line-search controller (CPU).

CG facts checked: agreement with both direct solves, local orthogonality of
residuals, monotone decrease of the A-norm error, finite termination on a grid
with few distinct eigenvalues. Line-search facts (Eqs. 12-13): exactness of
the step (new residual orthogonal to the direction), one-step convergence with
the exact error as the direction, the Jacobi direction reproducing
preconditioned steepest descent, and rejection of unusable directions.
"""
import numpy as np
import pytest

from paper_2604_01800_amd import inputs
from oracle import direct


def _problem(orc, n=48, beta=1.5, seed=0):
    g = inputs.make_grid(n, n, beta)
    b, _ = orc.rhs(g, inputs.gaussian_bumps(g, seed))
    return g, b


def test_pcg_matches_direct(orc):
    g, b = _problem(orc)
    xs = direct.separable_solve(g, b)
    for pc in (0, 1):
        x, st, _ = orc.pcg(g, b, precond=pc, tol=1e-12, max_iter=5000)
        assert st.converged
        x = x - x.mean()
        assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)


def test_pcg_residual_history_and_true_residual(orc):
    g, b = _problem(orc, 40, 2.0, 1)
    x, st, h = orc.pcg(g, b, tol=1e-8, max_iter=2000, history=True)
    assert st.converged and len(h) == st.iters_total + 1
    assert h[-1] <= 1e-8 * np.linalg.norm(b) and h[-2] > 1e-8 * np.linalg.norm(b)
    true = np.linalg.norm(b - orc.apply(g, x))
    assert abs(true - h[-1]) <= 1e-3 * h[-1] + 1e-14 * np.linalg.norm(b)


def _cg_iterates(orc, g, b, k):
    """Run 1..k fixed iterations (x0 = 0) through the oracle."""
    return [orc.pcg(g, b, tol=0, max_iter=m)[0] for m in range(1, k + 1)]


def test_cg_invariants(orc):
    g, b = _problem(orc, 24, 1.8, 2)
    d = orc.diag(g)
    xs = direct.separable_solve(g, b)
    xs_b = xs  # A^+ b
    xk = _cg_iterates(orc, g, b, 12)
    rs = [b - orc.apply(g, x) for x in xk]
    zs = [r / d for r in rs]
    # local orthogonality r_k^T z_j = 0 for consecutive iterates
    for k in range(1, len(rs)):
        rel = abs(np.sum(rs[k] * zs[k - 1])) / (np.linalg.norm(rs[k]) * np.linalg.norm(zs[k - 1]))
        assert rel < 1e-8
    # A-norm error is monotonically decreasing
    en = []
    for x in xk:
        e = (x - x.mean()) - xs_b
        en.append(np.sum(e * orc.apply(g, e)))
    assert all(en[k + 1] < en[k] for k in range(len(en) - 1))


def test_cg_finite_termination_uniform(orc):
    # 4x4 uniform grid: eigenvalues 4 sin^2(pi k/8) + 4 sin^2(pi l/8) take 9 distinct
    # nonzero values, so CG (no preconditioner; Jacobi is not a multiple of I
    # at the walls) terminates within 9 steps.
    g = inputs.make_grid(4, 4, 0.0)
    rng = np.random.default_rng(3)
    f = rng.standard_normal((4, 4))
    b, _ = orc.rhs(g, f)
    x, st, h = orc.pcg(g, b, precond=0, tol=1e-13, max_iter=50, history=True)
    assert st.converged and st.iters_total <= 9


def test_dlsm_exact_error_converges_in_one_step(orc):
    g, b = _problem(orc, 32, 1.5, 5)
    prov = lambda r: direct.separable_solve(g, r - r.mean())
    x, st, h = orc.hybrid(g, b, prov, tol=1e-10, max_iter=200, num_cg=3, num_dlsm=2, history=True)
    assert st.converged
    assert st.iters_cg == 3 and st.iters_dlsm == 1 and st.iters_total == 4


def test_dlsm_step_is_exact_line_search(orc):
    g, b = _problem(orc, 28, 2.0, 6)
    rng = np.random.default_rng(7)
    dirs = []

    def prov(r):
        e = rng.standard_normal(r.shape) + r
        dirs.append(e)
        return e

    x, st, h = orc.hybrid(g, b, prov, tol=0, max_iter=4, num_cg=3, num_dlsm=1)
    r = b - orc.apply(g, x)
    e = dirs[0]
    assert abs(np.sum(r * e)) <= 1e-11 * np.linalg.norm(r) * np.linalg.norm(e)


def test_dlsm_jacobi_direction_is_steepest_descent(orc):
    # With Num_CG-type = 0 and e = D^-1 r the hybrid is Jacobi-preconditioned
    # steepest descent: x <- x + (r.z / z.Az) z, z = D^-1 r.
    g, b = _problem(orc, 20, 1.2, 8)
    d = orc.diag(g)
    x, st, _ = orc.hybrid(g, b, lambda r: r / d, tol=0, max_iter=7, num_cg=0, num_dlsm=1)
    y = np.zeros_like(b)
    for _ in range(7):
        r = b - orc.apply(g, y)
        z = r / d
        y = y + np.sum(r * z) / np.sum(z * orc.apply(g, z)) * z
    np.testing.assert_allclose(x, y, rtol=1e-10, atol=1e-12 * np.abs(y).max())


def test_a_norm_error_monotone_across_blocks(orc):
    # CG steps, line-search steps and restarts never increase the A-norm error.
    # The provider is re-seeded per run, so run m is a prefix of run m + 1.
    g, b = _problem(orc, 24, 2.2, 9)
    xs = direct.separable_solve(g, b)
    traj = []
    for m in range(1, 16):
        rng = np.random.default_rng(12)
        prov = lambda r: r + 0.3 * rng.standard_normal(r.shape) * np.abs(r).max()
        x, _, _ = orc.hybrid(g, b, prov, tol=0, max_iter=m, num_cg=3, num_dlsm=2)
        e = (x - x.mean()) - xs
        traj.append(np.sum(e * orc.apply(g, e)))
    assert all(traj[k + 1] <= traj[k] * (1 + 1e-12) for k in range(len(traj) - 1)), traj


@pytest.mark.parametrize("kind", ["zero", "nan", "const"])
def test_unusable_directions_are_rejected(orc, kind):
    g, b = _problem(orc, 24, 1.5, 13)
    if kind == "zero":
        prov = lambda r: np.zeros_like(r)
    elif kind == "nan":
        prov = lambda r: np.full_like(r, np.nan)
    else:
        prov = lambda r: np.ones_like(r)  # null-space direction: e^T A e = 0
    x, st, h = orc.hybrid(g, b, prov, tol=1e-8, max_iter=20000, num_cg=3, num_dlsm=2, history=True)
    assert st.converged
    assert st.iters_dlsm == 0 and st.dlsm_rejected > 0
    assert np.linalg.norm(b - orc.apply(g, x)) <= 1.01e-8 * np.linalg.norm(b)


def test_iteration_totals_decompose_into_rounds(orc):
    # Every hybrid total is 5 * (full rounds) + remainder, with rounds starting
    # with CG (the paper's totals 9 = 5 + 4, 21 = 4 * 5 + 1, ...).
    g, b = _problem(orc, 32, 1.5, 14)
    prov = lambda r: direct.separable_solve(g, r - r.mean()) * (1 + 0.05 * np.cos(np.arange(r.size)).reshape(r.shape))
    x, st, h = orc.hybrid(g, b, prov, tol=1e-10, max_iter=500, num_cg=3, num_dlsm=2)
    full, rem = divmod(st.iters_total, 5)
    assert st.iters_cg == 3 * full + min(rem, 3)
    assert st.iters_dlsm == 2 * full + max(rem - 3, 0)
