"""Solid-mask operator (PPE_MASK_SOLID) on the GPU against the oracle's
solid-mask mode: only faces between two fluid cells carry flux, solid cells
hold identity rows, the right-hand side is projected over the fluid cells and
vanishes on solid cells.

Bars, as for the immersed-boundary operator: the FP32 stencil within 1e-6
relative (FP64 stencil 1e-13); fixed-k Jacobi-PCG and CG iterates within 1e-5
relative in x; converged solves judged on the oracle's FP64 true residual of
the masked system, with the solid cells untouched and the fluid mean zero."""
import numpy as np
import pytest
import torch
from scipy import ndimage

import oracle
from oracle import OGrid
from paper_2604_01800_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ppe():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_01800_amd import ppe as P
    P.lib()
    return P


def solid_system(nx, ny, seed, beta=None, params=None):
    rng = np.random.default_rng(seed)
    if beta is None:
        g = inputs.random_stretched_grid(nx, ny, rng)
    else:
        g = inputs.make_grid(nx, ny, beta, 0.8 * beta)
    if params is None:
        g = inputs.with_ellipse(g, rng)
    else:
        g.mask = inputs.ellipse_mask(g.xc, g.yc, params).astype(np.uint8)
    mask = np.asarray(g.mask).astype(np.uint8).reshape(ny, nx)
    g.mask = mask
    assert mask.any() and not mask.all()
    # one connected fluid region, so the null space is the fluid indicator
    _, ncomp = ndimage.label(mask == 0)
    assert ncomp == 1
    return g, inputs.grf(g, seed).astype(np.float32)


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def solve(ppe, prob, f, x0=None, **kw):
    f = np.asarray(f, dtype=np.float32)
    if f.ndim == 2:
        f = f[None]
    x = torch.zeros(f.shape, dtype=torch.float64, device="cuda") if x0 is None else dev(x0, torch.float64)
    st, stats = ppe.ppe_solve_plain(prob, dev(f, torch.float32), x, ppe.ppe_solve_opts_default(**kw))
    return st, stats, x.cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("nx,ny,beta", [(64, 64, 1.5), (70, 45, 2.0), (130, 67, 2.5), (200, 131, 1.2)])
def test_apply_matches_oracle(ppe, nx, ny, beta):
    g, _ = solid_system(nx, ny, nx + ny, beta=beta)
    og = OGrid(g, solid=True)
    prob = ppe.ppe_problem_create(g, mask_mode=ppe.PPE_MASK_SOLID)
    x = np.random.default_rng(3).standard_normal((3, ny, nx))
    x32 = x.astype(np.float32)
    y32 = torch.empty((3, ny, nx), dtype=torch.float32, device="cuda")
    y64 = torch.empty((3, ny, nx), dtype=torch.float64, device="cuda")
    ppe.ppe_apply_f32(prob, dev(x32, torch.float32), y32)
    ppe.ppe_apply_f64(prob, dev(x, torch.float64), y64)
    torch.cuda.synchronize()
    for s in range(3):
        r32 = oracle.apply(og, x32[s].astype(np.float64))
        r64 = oracle.apply(og, x[s])
        assert rel(y32[s].cpu().numpy(), r32) <= 1e-6
        assert rel(y64[s].cpu().numpy(), r64) <= 1e-13
        # identity rows on solid cells, bit-exact in FP64
        np.testing.assert_array_equal(y64[s].cpu().numpy()[g.mask == 1], x[s][g.mask == 1])
    # and the mask changes the operator: the default mode differs on the fluid next to the body
    assert rel(oracle.apply(g, x[0]), oracle.apply(og, x[0])) > 1e-3


@pytest.mark.parametrize("k", [1, 5, 17, 40])
@pytest.mark.parametrize("precond", [0, 1], ids=["cg", "jacobi"])
@pytest.mark.parametrize("nx,ny,beta", [(64, 64, 1.5), (130, 67, 2.5)])
def test_fixed_iterations_match_oracle(ppe, nx, ny, beta, precond, k):
    g, f = solid_system(nx, ny, 7, beta=beta)
    og = OGrid(g, solid=True)
    prob = ppe.ppe_problem_create(g, mask_mode=ppe.PPE_MASK_SOLID)
    st, stats, x = solve(ppe, prob, f, tol=0.0, max_iter=k, precond=precond)
    assert st == ppe.PPE_NOT_CONVERGED and stats[0]["iters_total"] == k
    b, mean = oracle.rhs(og, f)
    xo, so, _ = oracle.pcg(og, b, precond=precond, tol=0.0, max_iter=k)
    xo = oracle.remove_fluid_mean(g, xo)
    assert rel(x[0], xo) <= 1e-5
    assert np.all(x[0][g.mask == 1] == 0.0)
    assert abs(stats[0]["rhs_mean_removed"] - mean) <= 1e-12 * abs(mean) + 1e-300


def test_nonzero_start_on_solid_cells(ppe):
    """A start with values on solid cells: the identity rows drive them to
    zero, as in the oracle's iteration from the same start."""
    g, f = solid_system(96, 80, 11, beta=1.8)
    og = OGrid(g, solid=True)
    prob = ppe.ppe_problem_create(g, mask_mode=ppe.PPE_MASK_SOLID)
    x0 = np.random.default_rng(5).standard_normal((1, 80, 96))
    st, stats, x = solve(ppe, prob, f, x0=x0, tol=0.0, max_iter=12)
    b, _ = oracle.rhs(og, f)
    xo, _, _ = oracle.pcg(og, b, x0=x0[0], tol=0.0, max_iter=12)
    assert rel(x[0], oracle.remove_fluid_mean(g, xo)) <= 1e-5
    st, stats, x = solve(ppe, prob, f, x0=x0, tol=1e-8, max_iter=5000)
    assert st == ppe.PPE_OK
    # on a solid cell the residual is -x itself
    assert np.abs(x[0][g.mask == 1]).max() <= 1.001e-8 * np.linalg.norm(b)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("precond", [0, 1], ids=["cg", "jacobi"])
def test_converged_solves(ppe, seed, precond):
    g, f = solid_system(128, 96, 20 + seed)
    og = OGrid(g, solid=True)
    prob = ppe.ppe_problem_create(g, mask_mode=ppe.PPE_MASK_SOLID)
    b, _ = oracle.rhs(og, f)
    xs, so, _ = oracle.pcg(og, b, precond=1, tol=1e-13, max_iter=20000)
    assert so.converged
    xs = oracle.remove_fluid_mean(g, xs)
    for tol in (1e-6, 1e-8):
        st, stats, x = solve(ppe, prob, f, tol=tol, max_iter=20000, precond=precond)
        assert st == ppe.PPE_OK
        res = np.linalg.norm(b - oracle.apply(og, x[0])) / np.linalg.norm(b)
        assert res <= tol * 1.001, (res, stats[0])
        assert abs(res - stats[0]["rel_res_true"]) <= 1e-3 * res
        assert np.all(x[0][g.mask == 1] == 0.0)
        assert abs(x[0][g.mask == 0].mean()) <= 1e-12 * np.abs(x[0]).max()
        if tol == 1e-8:
            assert rel(x[0], xs) <= 1e-5
    if precond == 1:
        _, s6, _ = oracle.pcg(og, b, precond=1, tol=1e-8, max_iter=20000)
        assert s6.iters_total - 3 <= stats[0]["iters_total"] <= 1.3 * s6.iters_total + 3


def test_batched_equals_single(ppe):
    g, _ = solid_system(100, 70, 41, beta=2.0)
    prob = ppe.ppe_problem_create(g, mask_mode=ppe.PPE_MASK_SOLID)
    fs = np.stack([inputs.grf(g, 300 + k).astype(np.float32) for k in range(3)])
    st, stats, xb = solve(ppe, prob, fs, tol=1e-7)
    assert st == ppe.PPE_OK
    for k in range(3):
        st1, s1, x1 = solve(ppe, prob, fs[k], tol=1e-7)
        np.testing.assert_array_equal(x1[0], xb[k])
        assert s1[0]["iters_total"] == stats[k]["iters_total"]


def test_history_matches_oracle(ppe):
    g, f = solid_system(64, 64, 9, beta=1.5)
    og = OGrid(g, solid=True)
    b, _ = oracle.rhs(og, f)
    _, so, ho = oracle.pcg(og, b, precond=1, tol=1e-7, max_iter=5000, history=True)
    prob = ppe.ppe_problem_create(g, mask_mode=ppe.PPE_MASK_SOLID)
    st, stats, x = solve(ppe, prob, f, tol=1e-7, record_history=1)
    assert st == ppe.PPE_OK
    h = stats[0]["history"]
    assert len(h) == stats[0]["iters_total"] + 1 == stats[0]["history_len"]
    assert h[0] == pytest.approx(1.0, rel=1e-6)
    assert h[-1] <= 1e-7 * 1.001 and h[-1] == pytest.approx(stats[0]["rel_res_true"], rel=1e-12)
    m = min(20, len(h), len(ho))
    np.testing.assert_allclose(h[:m], ho[:m] / np.linalg.norm(b), rtol=1e-3)


def test_full_size_1024(ppe):
    """1024^2, random stretching and an ellipse, Jacobi-PCG to 1e-6."""
    g, f = solid_system(1024, 1024, 61)
    og = OGrid(g, solid=True)
    prob = ppe.ppe_problem_create(g, mask_mode=ppe.PPE_MASK_SOLID)
    st, stats, x = solve(ppe, prob, f, tol=1e-6, max_iter=50000)
    assert st == ppe.PPE_OK
    b, _ = oracle.rhs(og, f)
    res = np.linalg.norm(b - oracle.apply(og, x[0])) / np.linalg.norm(b)
    print(f"solid-mask 1024^2: {stats[0]['iters_total']} iterations, {stats[0]['ms_total']:.1f} ms, rel res {res:.2e}")
    assert res <= 1e-6 * 1.001
    assert np.all(x[0][g.mask == 1] == 0.0)


def test_unsupported_paths(ppe):
    g, f = solid_system(64, 64, 2, beta=1.5)
    prob = ppe.ppe_problem_create(g, mask_mode=ppe.PPE_MASK_SOLID)
    fd = dev(f[None], torch.float32)
    x = torch.zeros((1, 64, 64), dtype=torch.float64, device="cuda")

    def unsupported(fn, *a, **kw):
        with pytest.raises(ppe.PPEError) as e:
            fn(*a, **kw)
        assert e.value.status == ppe.PPE_ERR_UNSUPPORTED, e.value

    unsupported(ppe.ppe_solve_plain, prob, fd, x, ppe.ppe_solve_opts_default(precond=ppe.PPE_PC_MG))
    unsupported(ppe.ppe_solve_hybrid, prob, None, fd, x, ppe.ppe_solve_opts_default(direction=ppe.PPE_DIR_ONES))
    unsupported(ppe.ppe_solve_plain_noalloc, prob, fd[0], x[0])
    unsupported(ppe.ppe_solve_batch, [prob], [fd[0]], [x[0]])
    unsupported(ppe.ppe_apply_precond, prob, fd, torch.empty_like(fd))
    unsupported(ppe.ppe_profile_pcg, prob, fd, x, reps=1)
    unsupported(ppe.ppe_generate_rhs, [prob], ppe.ppe_train_opts_default(), torch.empty_like(fd))
    # a mask is required, and a mask with no fluid cell is refused
    with pytest.raises(ppe.PPEError):
        ppe.ppe_problem_create(inputs.make_grid(8, 8, 1.0), mask_mode=ppe.PPE_MASK_SOLID)
    gs = inputs.make_grid(8, 8, 1.0)
    gs.mask = np.ones((8, 8), np.uint8)
    with pytest.raises(ppe.PPEError):
        ppe.ppe_problem_create(gs, mask_mode=ppe.PPE_MASK_SOLID)
