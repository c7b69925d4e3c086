"""Incomplete-Cholesky PCG (the ICPCG CG-type of Sec. 2.5, IC(0) in
red-black ordering) on the GPU against the FP64 oracle (oracle.ic): one
application against the oracle's triangular solves, fixed-k ICPCG iterates
against the oracle's PCG with the same preconditioner, converged solves
judged on the oracle's FP64 true residual, the hybrid over ICPCG against the
oracle hybrid, the 1024^2 benchmark system, and the argument checks.

Bars. One application is two FP32 passes (a few roundings per cell, no
cancellation: the operator is an M-matrix), so 1e-6 relative against the
FP64 triangular solves; CG iterates after up to 20 iterations within 2e-5,
as for Jacobi-PCG (1e-5) with the extra passes' rounding."""
import numpy as np
import pytest
import torch

import oracle
from oracle import ic as oic
from paper_2604_01800_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ppe():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_01800_amd import ppe as P
    P.lib()
    return P


def system(nx, ny, seed, beta=None):
    rng = np.random.default_rng(seed)
    g = inputs.random_stretched_grid(nx, ny, rng) if beta is None else inputs.make_grid(nx, ny, beta, 0.7 * beta)
    return g, inputs.grf(g, seed).astype(np.float32)


def true_res(g, f, x):
    b, _ = oracle.rhs(g, f)
    return np.linalg.norm(b - oracle.apply(g, x)) / np.linalg.norm(b)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def ic_opts(ppe, **kw):
    return ppe.ppe_solve_opts_default(precond=ppe.PPE_PC_IC, **kw)


@pytest.mark.parametrize("nx,ny", [(64, 48), (70, 45), (130, 67), (2, 2), (3, 130), (200, 9)])
def test_apply_matches_oracle(ppe, nx, ny):
    g, _ = system(nx, ny, nx + ny)
    P = oic.RedBlackIC(g)
    prob = ppe.ppe_problem_create(g)
    r = np.random.default_rng(2).standard_normal((2, ny, nx)).astype(np.float32)
    z = torch.zeros((2, ny, nx), dtype=torch.float32, device="cuda")
    ppe.ppe_apply_precond(prob, torch.from_numpy(r).cuda(), z, ic_opts(ppe))
    for k in range(2):
        want = P.apply(r[k].astype(np.float64))
        assert rel(z[k].cpu().numpy().astype(np.float64), want) <= 1e-6


@pytest.mark.parametrize("k", [1, 2, 5, 20])
def test_fixed_iterations_match_oracle(ppe, k):
    g, f = system(96, 64, 5)
    P = oic.RedBlackIC(g)
    b, _ = oracle.rhs(g, f)
    xo, so, _ = oracle.pcg(g, b, precond=2, pc=P.apply, tol=0.0, max_iter=k)
    prob = ppe.ppe_problem_create(g)
    x = torch.zeros((1, 64, 96), dtype=torch.float64, device="cuda")
    st, s = ppe.ppe_solve_plain(prob, torch.from_numpy(f[None]).cuda(), x, ic_opts(ppe, tol=0.0, max_iter=k))
    assert st == ppe.PPE_NOT_CONVERGED and s[0]["iters_total"] == k
    xg = x[0].cpu().numpy()
    assert rel(xg - xg.mean(), xo - xo.mean()) <= 2e-5


@pytest.mark.parametrize("nx,ny,tol", [(64, 64, 1e-6), (128, 96, 1e-8), (200, 131, 1e-6)])
def test_converged_solves(ppe, nx, ny, tol):
    g, f = system(nx, ny, 6)
    prob = ppe.ppe_problem_create(g)
    x = torch.zeros((1, ny, nx), dtype=torch.float64, device="cuda")
    st, s = ppe.ppe_solve_plain(prob, torch.from_numpy(f[None]).cuda(), x, ic_opts(ppe, tol=tol, max_iter=20000))
    assert st == ppe.PPE_OK
    xg = x[0].cpu().numpy()
    res = true_res(g, f, xg)
    assert res <= tol * 1.001 and abs(res - s[0]["rel_res_true"]) <= 1e-3 * res
    assert abs(xg.mean()) <= 1e-12 * np.abs(xg).max()
    b, _ = oracle.rhs(g, f)
    _, so, _ = oracle.pcg(g, b, precond=2, pc=oic.RedBlackIC(g).apply, tol=tol, max_iter=20000)
    _, sj, _ = oracle.pcg(g, b, precond=1, tol=tol, max_iter=20000)
    print(f"{nx}x{ny} tol {tol:g}: ICPCG GPU {s[0]['iters_total']}, oracle {so.iters_total}, "
          f"oracle Jacobi-PCG {sj.iters_total}")
    assert so.iters_total - 3 <= s[0]["iters_total"] <= 1.2 * so.iters_total + 3
    assert so.iters_total < sj.iters_total


def test_batched_equals_single_and_graph_equals_eager(ppe):
    g, _ = system(96, 64, 7)
    fs = np.stack([inputs.grf(g, 70 + k).astype(np.float32) for k in range(3)])
    prob = ppe.ppe_problem_create(g)
    o = ic_opts(ppe, tol=1e-7)
    x = torch.zeros((3, 64, 96), dtype=torch.float64, device="cuda")
    st, s = ppe.ppe_solve_plain(prob, torch.from_numpy(fs).cuda(), x, o)
    assert st == ppe.PPE_OK
    for k in range(3):
        x1 = torch.zeros((1, 64, 96), dtype=torch.float64, device="cuda")
        ppe.ppe_solve_plain(prob, torch.from_numpy(fs[k:k + 1]).cuda(), x1, o)
        np.testing.assert_array_equal(x1[0].cpu().numpy(), x[k].cpu().numpy())
    x2 = torch.zeros_like(x)
    o.use_graph = 0
    ppe.ppe_solve_plain(prob, torch.from_numpy(fs).cuda(), x2, o)
    np.testing.assert_array_equal(x.cpu().numpy(), x2.cpu().numpy())


def test_history_matches_oracle(ppe):
    g, f = system(64, 48, 10)
    b, _ = oracle.rhs(g, f)
    _, so, ho = oracle.pcg(g, b, precond=2, pc=oic.RedBlackIC(g).apply, tol=1e-6, max_iter=2000, history=True)
    prob = ppe.ppe_problem_create(g)
    x = torch.zeros((1, 48, 64), dtype=torch.float64, device="cuda")
    st, s = ppe.ppe_solve_plain(prob, torch.from_numpy(f[None]).cuda(), x, ic_opts(ppe, tol=1e-6, record_history=1))
    h = s[0]["history"]
    assert st == ppe.PPE_OK and len(h) == s[0]["iters_total"] + 1
    m = min(20, len(h), len(ho))
    np.testing.assert_allclose(h[:m], ho[:m] / np.linalg.norm(b), rtol=1e-3)


def test_hybrid_over_ic_matches_oracle(ppe):
    """DLSM over ICPCG (the paper's HyDEA with its ICPCG CG-type), the
    Jacobi direction standing in for the network: iterates after a fixed
    count against the oracle hybrid with the oracle IC(0)."""
    g, f = system(64, 64, 8)
    P = oic.RedBlackIC(g)
    b, _ = oracle.rhs(g, f)
    d = oracle.diag(g)
    prob = ppe.ppe_problem_create(g)
    for k in (5, 12):
        xo, so, _ = oracle.hybrid(g, b, lambda r: r / d, precond=2, pc=P.apply, tol=0.0, max_iter=k)
        x = torch.zeros((1, 64, 64), dtype=torch.float64, device="cuda")
        st, s = ppe.ppe_solve_hybrid(prob, None, torch.from_numpy(f[None]).cuda(), x,
                                     ic_opts(ppe, tol=0.0, max_iter=k, direction=ppe.PPE_DIR_JACOBI))
        assert s[0]["iters_total"] == k and s[0]["iters_dlsm"] == so.iters_dlsm
        xg = x[0].cpu().numpy()
        assert rel(xg - xg.mean(), xo - xo.mean()) <= 2e-5
    x = torch.zeros((1, 64, 64), dtype=torch.float64, device="cuda")
    st, s = ppe.ppe_solve_hybrid(prob, None, torch.from_numpy(f[None]).cuda(), x,
                                 ic_opts(ppe, tol=1e-6, max_iter=20000, direction=ppe.PPE_DIR_JACOBI))
    assert st == ppe.PPE_OK and true_res(g, f, x[0].cpu().numpy()) <= 1e-6 * 1.001


def test_full_size_1024_ic(ppe):
    """The benchmark system (1024^2, beta 1.75, ellipse, GRF): ICPCG
    converges on the FP64 true residual in fewer iterations than Jacobi-PCG
    (about 5 600 at this size)."""
    g = inputs.with_ellipse(inputs.make_grid(1024, 1024, 1.75), np.random.default_rng(0))
    f = inputs.grf(g, 0).astype(np.float32)
    prob = ppe.ppe_problem_create(g)
    x = torch.zeros((1, 1024, 1024), dtype=torch.float64, device="cuda")
    st, s = ppe.ppe_solve_plain(prob, torch.from_numpy(f[None]).cuda(), x, ic_opts(ppe, tol=1e-6, max_iter=20000))
    assert st == ppe.PPE_OK
    res = true_res(g, f, x[0].cpu().numpy())
    print(f"1024^2 ICPCG: {s[0]['iters_total']} iterations, {s[0]['ms_total']:.1f} ms, true rel res {res:.2e}")
    assert res <= 1e-6 * 1.001 and s[0]["iters_total"] < 5000


def test_ic_argument_checks(ppe):
    g, f = system(48, 32, 9)
    prob = ppe.ppe_problem_create(g)
    fd = torch.from_numpy(f[None]).cuda()
    x = torch.zeros((1, 32, 48), dtype=torch.float64, device="cuda")
    with pytest.raises(ppe.PPEError) as e:  # one-cell-wide grids: IC(0) breaks down
        g1 = inputs.make_grid(40, 1, 1.0)
        ppe.ppe_solve_plain(ppe.ppe_problem_create(g1), torch.zeros((1, 1, 40), device="cuda"),
                            torch.zeros((1, 1, 40), dtype=torch.float64, device="cuda"), ic_opts(ppe))
    assert e.value.status == ppe.PPE_ERR_SHAPE
    for call in (lambda: ppe.ppe_solve_batch([prob], [fd[0]], [x[0]], ic_opts(ppe)),
                 lambda: ppe.ppe_solve_plain_noalloc(prob, fd[0], x[0], ic_opts(ppe))):
        with pytest.raises(ppe.PPEError) as e:
            call()
        assert e.value.status == ppe.PPE_ERR_UNSUPPORTED
    gs = inputs.with_ellipse(inputs.make_grid(48, 32, 1.2), np.random.default_rng(1))
    ps = ppe.ppe_problem_create(gs, mask_mode=ppe.PPE_MASK_SOLID)
    with pytest.raises(ppe.PPEError) as e:
        ppe.ppe_solve_plain(ps, fd, x, ic_opts(ppe))
    assert e.value.status == ppe.PPE_ERR_UNSUPPORTED
