"""Mixed-size batches (one launch per two iterations, or per iteration, over a
work list of all grids) against single solves and the oracle: every solve of
the batch is bit-identical to the same solve alone (same iteration form and
tile height: identical arithmetic and reduction order), reaches the tolerance
on the FP64 true residual the oracle recomputes, and keeps its own status and
timing. With a network the batch runs hybrid solves, each bit-identical to
the same hybrid solve alone."""
import numpy as np
import pytest
import torch

import oracle
from paper_2604_01800_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ppe():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_01800_amd import ppe as P
    P.lib()
    return P


def systems(shapes, seed):
    rng = np.random.default_rng(seed)
    out = []
    for k, (nx, ny) in enumerate(shapes):
        g = inputs.with_ellipse(inputs.random_stretched_grid(nx, ny, rng), rng)
        out.append((g, inputs.grf(g, seed * 100 + k).astype(np.float32)))
    return out


def run_batch(ppe, sys_, **kw):
    probs = [ppe.ppe_problem_create(g) for g, _ in sys_]
    fs = [torch.from_numpy(f).cuda() for _, f in sys_]
    xs = [torch.zeros(f.shape, dtype=torch.float64, device="cuda") for _, f in sys_]
    st, stats = ppe.ppe_solve_batch(probs, fs, xs, ppe.ppe_solve_opts_default(**kw))
    return st, stats, [x.cpu().numpy() for x in xs], probs


def true_res(g, f, x):
    b, _ = oracle.rhs(g, f)
    return np.linalg.norm(b - oracle.apply(g, x)) / np.linalg.norm(b)


@pytest.mark.parametrize("variant,rows", [(3, 4), (3, 20), (1, 4)], ids=["two_step_R4", "two_step_R20", "single_R4"])
def test_mixed_batch_equals_single_solves(ppe, variant, rows):
    sys_ = systems([(130, 67), (64, 64), (200, 150), (96, 256), (33, 21)], seed=1)
    st, stats, xs, probs = run_batch(ppe, sys_, tol=1e-7, rows_per_wave=rows, variant=variant)
    assert st == ppe.PPE_OK
    for (g, f), x, s, p in zip(sys_, xs, stats, probs):
        assert true_res(g, f, x) <= 1e-7 * 1.001
        assert abs(x.mean()) <= 1e-12 * np.abs(x).max()
        fd = torch.from_numpy(f[None]).cuda()
        xd = torch.zeros((1,) + f.shape, dtype=torch.float64, device="cuda")
        st1, s1 = ppe.ppe_solve_plain(p, fd, xd, ppe.ppe_solve_opts_default(
            tol=1e-7, rows_per_wave=rows, variant=variant))
        assert st1 == ppe.PPE_OK and s1[0]["iters_total"] == s["iters_total"]
        np.testing.assert_array_equal(xd[0].cpu().numpy(), x)
        assert 0.0 < s["ms_device"] <= s["ms_total"]


def test_batch_statuses_are_per_solve(ppe):
    sys_ = systems([(48, 40), (64, 32), (40, 40)], seed=2)
    bad = sys_[1][1].copy()
    bad[3, 5] = np.nan
    sys_[1] = (sys_[1][0], bad)
    st, stats, xs, _ = run_batch(ppe, sys_, tol=1e-6)
    assert st == ppe.PPE_ERR_NONFINITE
    assert [s["status"] for s in stats] == [ppe.PPE_OK, ppe.PPE_ERR_NONFINITE, ppe.PPE_OK]
    for k in (0, 2):
        assert true_res(sys_[k][0], sys_[k][1], xs[k]) <= 1e-6 * 1.001
    # iteration limit: only the solve that needs more iterations stops short
    sys_ = systems([(32, 32), (256, 256)], seed=3)
    st, stats, xs, _ = run_batch(ppe, sys_, tol=1e-6, max_iter=300)
    assert st == ppe.PPE_NOT_CONVERGED
    assert stats[0]["status"] == ppe.PPE_OK and stats[1]["status"] == ppe.PPE_NOT_CONVERGED
    assert stats[1]["iters_total"] == 300
    assert abs(true_res(sys_[1][0], sys_[1][1], xs[1]) - stats[1]["rel_res_true"]) <= 1e-6 * stats[1]["rel_res_true"]


def test_uneven_grids_workload(ppe):
    """Twelve grids between 128^2 and 1024^2 (ellipse masks, GRF sources) in one
    batch to 1e-6: every solve converges on the oracle's true residual; small
    grids finish first on the device clock; aggregate rate printed."""
    rng = np.random.default_rng(4)
    sizes = [128, 256, 384, 512, 768, 1024]
    shapes = [(int(rng.choice(sizes)), int(rng.choice(sizes))) for _ in range(12)]
    sys_ = systems(shapes, seed=4)
    st, stats, xs, _ = run_batch(ppe, sys_, tol=1e-6)
    assert st == ppe.PPE_OK
    for (g, f), x in zip(sys_, xs):
        assert true_res(g, f, x) <= 1e-6 * 1.001
    cells = [nx * ny for nx, ny in shapes]
    small, large = int(np.argmin(cells)), int(np.argmax(cells))
    assert stats[small]["ms_device"] < stats[large]["ms_device"]
    print("uneven batch of %d grids: %.1f ms wall, %.2f solves/s; per-solve device ms %s" % (
        len(shapes), stats[0]["ms_total"], 1e3 * len(shapes) / stats[0]["ms_total"],
        [round(s["ms_device"], 1) for s in stats]))


def test_batch_argument_checks(ppe):
    sys_ = systems([(32, 32)], seed=5)
    p = ppe.ppe_problem_create(sys_[0][0])
    f = torch.from_numpy(sys_[0][1]).cuda()
    x = torch.zeros(f.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(ppe.PPEError):  # the same problem twice
        ppe.ppe_solve_batch([p, p], [f, f], [x, x.clone()])
    with pytest.raises(ValueError):
        ppe.ppe_solve_batch([p], [f[:16]], [x])
    with pytest.raises(ppe.PPEError):  # the two-phase form is not batched over mixed sizes
        ppe.ppe_solve_batch([p], [f], [x], ppe.ppe_solve_opts_default(variant=ppe.PPE_PCG_TWO_PHASE))
    assert ppe.lib().ppe_solve_batch(0, None, None, None, None, None, None, None) == ppe.PPE_OK


# Hybrid solves of a mixed-size batch: the rounds of every solve advance in
# lock step, and each solve is bit-identical to the same hybrid solve alone
# (same kernels, arguments and order on its own buffers).
HYB_SHAPES = [(64, 64), (128, 72), (40, 96), (32, 32)]  # multiples of 8 for the 4-level network


def _single_hybrid(ppe, p, net, f, **kw):
    fd = torch.from_numpy(f[None]).cuda()
    xd = torch.zeros((1,) + f.shape, dtype=torch.float64, device="cuda")
    st, s = ppe.ppe_solve_hybrid(p, net, fd, xd, ppe.ppe_solve_opts_default(**kw))
    return st, s[0], xd[0].cpu().numpy()


# With the network direction the forwards of the batch run as one grouped
# launch per layer; the solves decide at different rounds in the "to_tol"
# cases (a loose tolerance: the random-init network's hybrid is a restarted
# CG(3) and slow to reach a tight one), so the grouped replay unit is rebuilt
# for fewer solves on the way and decided solves skip their share of the
# grouped launches.
@pytest.mark.parametrize("direction,tol,max_iter,graph", [(2, 1e-6, 20000, 1), (0, 0.0, 23, 1), (0, 0.0, 40, 1),
                                                          (0, 1e-2, 20000, 1), (0, 1e-2, 20000, 0)],
                         ids=["jacobi_to_tol", "net_23_iters", "net_40_iters", "net_to_tol", "net_to_tol_eager"])
def test_hybrid_mixed_batch_equals_single_solves(ppe, direction, tol, max_iter, graph):
    sys_ = systems(HYB_SHAPES, seed=4)
    net = ppe.Net(ppe.ppe_net_config_default(), seed=3)
    probs = [ppe.ppe_problem_create(g) for g, _ in sys_]
    fs = [torch.from_numpy(f).cuda() for _, f in sys_]
    xs = [torch.zeros(f.shape, dtype=torch.float64, device="cuda") for _, f in sys_]
    kw = dict(tol=tol, max_iter=max_iter, direction=direction, use_graph=graph)
    st, stats = ppe.ppe_solve_batch(probs, fs, xs, ppe.ppe_solve_opts_default(**kw), net=net)
    assert st == (ppe.PPE_OK if tol > 0 else ppe.PPE_NOT_CONVERGED)
    for (g, f), x, s, p in zip(sys_, xs, stats, probs):
        st1, s1, x1 = _single_hybrid(ppe, p, net, f, **kw)
        np.testing.assert_array_equal(x.cpu().numpy(), x1)
        for k in ("status", "iters_total", "iters_cg", "iters_dlsm", "dlsm_rejected", "reliable_updates"):
            assert s[k] == s1[k], (k, s, s1)
        if tol > 0:
            assert s["status"] == ppe.PPE_OK
            assert true_res(g, f, x.cpu().numpy()) <= tol * 1.001
        else:
            assert s["iters_total"] == max_iter and s["iters_dlsm"] > 0
    if direction == 0 and tol > 0:  # the solves decided at different rounds
        print("iterations", [s["iters_total"] for s in stats])
        assert len({s["iters_total"] for s in stats}) > 1


# The grouped forward: shapes whose coarse levels split their K loop (the
# small grids) next to ones that do not, both local-weight forms and none.
FWD_SHAPES = [(64, 64), (128, 72), (40, 96), (32, 32), (256, 200), (16, 24)]


# More than 2^22 cells in all: the grids are packed into two parts.
FWD_SHAPES_LARGE = [(2048, 1536), (64, 64), (1024, 1040), (640, 384), (128, 128), (40, 96)]


@pytest.mark.parametrize("use_eta,shapes", [(2, FWD_SHAPES), (1, FWD_SHAPES), (0, FWD_SHAPES), (2, FWD_SHAPES_LARGE)],
                         ids=["per_node", "per_channel", "no_eta", "per_node_parts"])
def test_forward_batch_equals_single_forwards(ppe, use_eta, shapes):
    net = ppe.Net(ppe.ppe_net_config_default(use_eta=use_eta), seed=5)
    sys_ = systems(shapes, seed=8)
    probs = [ppe.ppe_problem_create(g) for g, _ in sys_]
    rs = [torch.from_numpy(f).cuda() for _, f in sys_]
    ys = [torch.full(f.shape, float("nan"), dtype=torch.float32, device="cuda") for _, f in sys_]
    ppe.ppe_net_forward_batch(net, probs, rs, ys)
    for p, r, y in zip(probs, rs, ys):
        y1 = torch.zeros((1,) + tuple(r.shape), dtype=torch.float32, device="cuda")
        ppe.ppe_net_forward(net, p, r[None], y1)
        np.testing.assert_array_equal(y.cpu().numpy(), y1[0].cpu().numpy())
        assert torch.isfinite(y).all()
    # order within the batch does not matter, and a single member is the plain forward
    ys2 = [torch.zeros_like(y) for y in ys]
    ppe.ppe_net_forward_batch(net, probs[::-1], rs[::-1], ys2[::-1])
    for y, y2 in zip(ys, ys2):
        assert torch.equal(y, y2)
    y3 = torch.zeros_like(ys[2])
    ppe.ppe_net_forward_batch(net, [probs[2]], [rs[2]], [y3])
    assert torch.equal(y3, ys[2])


def test_forward_batch_with_tuned_members(ppe):
    """Grids whose forward was tile-width tuned keep, inside the grouped
    launch, the K split of their own tuned width: still bit-identical."""
    net = ppe.Net(ppe.ppe_net_config_default(), seed=5)
    sys_ = systems(FWD_SHAPES, seed=9)
    probs = [ppe.ppe_problem_create(g) for g, _ in sys_]
    for k in (0, 4):
        ppe.ppe_tune_net(net, probs[k], nb=1, reps=3)
    rs = [torch.from_numpy(f).cuda() for _, f in sys_]
    ys = [torch.zeros_like(r) for r in rs]
    ppe.ppe_net_forward_batch(net, probs, rs, ys)
    for p, r, y in zip(probs, rs, ys):
        y1 = torch.zeros((1,) + tuple(r.shape), dtype=torch.float32, device="cuda")
        ppe.ppe_net_forward(net, p, r[None], y1)
        np.testing.assert_array_equal(y.cpu().numpy(), y1[0].cpu().numpy())


def test_forward_batch_checks(ppe):
    net = ppe.Net(ppe.ppe_net_config_default(), seed=5)
    sys_ = systems(FWD_SHAPES[:2], seed=8)
    probs = [ppe.ppe_problem_create(g) for g, _ in sys_]
    rs = [torch.from_numpy(f).cuda() for _, f in sys_]
    ys = [torch.zeros_like(r) for r in rs]
    with pytest.raises(ppe.PPEError) as e:  # the same problem twice
        ppe.ppe_net_forward_batch(net, [probs[0], probs[0]], [rs[0], rs[0]], [ys[0], ys[0]])
    assert e.value.status == ppe.PPE_ERR_INVALID_ARG
    g36 = inputs.make_grid(36, 36, 1.5)
    with pytest.raises(ppe.PPEError) as e:  # 36 is not divisible by 8
        ppe.ppe_net_forward_batch(net, [probs[0], ppe.ppe_problem_create(g36)],
                                  [rs[0], torch.zeros((36, 36), device="cuda")],
                                  [ys[0], torch.zeros((36, 36), device="cuda")])
    assert e.value.status == ppe.PPE_ERR_SHAPE
    ppe.ppe_net_forward_batch(net, [], [], [])


def test_hybrid_batch_statuses_and_checks(ppe):
    sys_ = systems(HYB_SHAPES[:3], seed=6)
    net = ppe.Net(ppe.ppe_net_config_default(), seed=3)
    probs = [ppe.ppe_problem_create(g) for g, _ in sys_]
    fs = [torch.from_numpy(f).cuda() for _, f in sys_]
    fs[1][3, 5] = float("nan")
    xs = [torch.zeros(f.shape, dtype=torch.float64, device="cuda") for _, f in sys_]
    o = ppe.ppe_solve_opts_default(tol=1e-6, max_iter=20000, direction=ppe.PPE_DIR_JACOBI)
    st, stats = ppe.ppe_solve_batch(probs, fs, xs, o, net=net)
    assert st == ppe.PPE_ERR_NONFINITE
    assert [s["status"] for s in stats] == [ppe.PPE_OK, ppe.PPE_ERR_NONFINITE, ppe.PPE_OK]
    for (g, f), x, s in zip(sys_, xs, stats):
        if s["status"] == ppe.PPE_OK:
            assert true_res(g, f, x.cpu().numpy()) <= 1e-6 * 1.001
    # a grid the 4-level network cannot pool is rejected when the network is used
    g36 = inputs.make_grid(36, 36, 1.5)
    p36 = ppe.ppe_problem_create(g36)
    f36 = torch.zeros((36, 36), dtype=torch.float32, device="cuda")
    x36 = torch.zeros((36, 36), dtype=torch.float64, device="cuda")
    with pytest.raises(ppe.PPEError):
        ppe.ppe_solve_batch([probs[0], p36], [fs[0], f36], [xs[0], x36], ppe.ppe_solve_opts_default(), net=net)
    with pytest.raises(ppe.PPEError):  # the same problem twice
        ppe.ppe_solve_batch([probs[0], probs[0]], [fs[0], fs[0]], [xs[0], xs[0].clone()], o, net=net)


def test_batch_after_destroyed_problems_of_other_sizes(ppe):
    """Batches on freshly created problems after the previous batch's problems
    were destroyed: the allocator may hand the new handles the old addresses
    (in the same order), yet the work list must follow the new grids. Each
    solve is judged on the oracle's true residual."""
    import gc
    for shapes in ([(64, 64), (96, 40)], [(200, 130), (150, 210)], [(40, 24), (33, 47)]):
        sys_ = systems(shapes, seed=7)
        st, stats, xs, probs = run_batch(ppe, sys_, tol=1e-7)
        assert st == ppe.PPE_OK
        for (g, f), x in zip(sys_, xs):
            assert true_res(g, f, x) <= 1e-7 * 1.001
        del probs
        gc.collect()
