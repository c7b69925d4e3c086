"""GPU parity of the hybrid PCG / line-search solve (Sec. 2.2, Eqs. 12-13).

* With the Jacobi direction e = D^-1 r standing in for the network, the GPU
  iterates (FP32 vectors, FP64 sums) match the oracle's FP64 hybrid iteration
  by iteration (relative 1e-5 in x after k iterations).
* Unusable directions (zero, NaN, null-space ones) are rejected and the solve
  still converges; the rejected steps are counted.
* With the network, one full round matches the oracle (FP64 network with the
  same BF16 weights) within the network's BF16 error, and full solves reach
  the tolerance on the FP64 true residual recomputed by the oracle.
"""
import numpy as np
import pytest
import torch

from paper_2604_01800_amd import inputs
from oracle import direct
from oracle import net as onet

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ppe():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_01800_amd import ppe as P
    P.lib()
    return P


def _solve(ppe, prob, net, f, **kw):
    f = np.asarray(f, np.float32)
    if f.ndim == 2:
        f = f[None]
    fd = torch.from_numpy(f).cuda()
    x = torch.zeros(f.shape, dtype=torch.float64, device="cuda")
    st, stats = ppe.ppe_solve_hybrid(prob, net, fd, x, ppe.ppe_solve_opts_default(**kw))
    return st, stats, x.cpu().numpy()


@pytest.mark.parametrize("k", [1, 3, 4, 5, 6, 9, 13])
@pytest.mark.parametrize("nx,ny,beta", [(48, 40, 1.5), (70, 33, 2.2)])
def test_jacobi_direction_matches_oracle(ppe, orc, k, nx, ny, beta):
    g = inputs.make_grid(nx, ny, beta)
    prob = ppe.ppe_problem_create(g)
    f = inputs.gaussian_bumps(g, 3).astype(np.float32)
    st, stats, x = _solve(ppe, prob, None, f, tol=0.0, max_iter=k, direction=ppe.PPE_DIR_JACOBI)
    assert stats[0]["iters_total"] == k
    b, _ = orc.rhs(g, f)
    d = orc.diag(g)
    xo, so, _ = orc.hybrid(g, b, lambda r: r / d, tol=0.0, max_iter=k, num_cg=3, num_dlsm=2)
    assert stats[0]["iters_cg"] == so.iters_cg and stats[0]["iters_dlsm"] == so.iters_dlsm
    xo = orc.remove_mean(xo)
    assert np.linalg.norm(x[0] - xo) / np.linalg.norm(xo) <= 1e-5


@pytest.mark.parametrize("ncg,ndl", [(3, 2), (1, 1), (2, 3), (0, 2), (5, 1)])
def test_jacobi_direction_round_shapes(ppe, orc, ncg, ndl):
    g = inputs.make_grid(40, 40, 1.8)
    prob = ppe.ppe_problem_create(g)
    f = inputs.gaussian_bumps(g, 4).astype(np.float32)
    k = 3 * (ncg + ndl) + 1
    st, stats, x = _solve(ppe, prob, None, f, tol=0.0, max_iter=k, num_cg=ncg, num_dlsm=ndl,
                          direction=ppe.PPE_DIR_JACOBI)
    b, _ = orc.rhs(g, f)
    d = orc.diag(g)
    xo, so, _ = orc.hybrid(g, b, lambda r: r / d, tol=0.0, max_iter=k, num_cg=ncg, num_dlsm=ndl)
    assert stats[0]["iters_total"] == so.iters_total
    assert np.linalg.norm(x[0] - orc.remove_mean(xo)) / np.linalg.norm(xo) <= 1e-5


@pytest.mark.parametrize("direction", ["ZERO", "NAN", "ONES"])
def test_rejected_directions_fall_back_to_pcg(ppe, orc, direction):
    g = inputs.make_grid(40, 32, 1.5)
    prob = ppe.ppe_problem_create(g)
    f = inputs.gaussian_bumps(g, 5).astype(np.float32)
    code = getattr(ppe, "PPE_DIR_" + direction)
    st, stats, x = _solve(ppe, prob, None, f, tol=1e-7, max_iter=20000, direction=code)
    assert st == ppe.PPE_OK
    s0 = stats[0]
    assert s0["iters_dlsm"] == 0 and s0["dlsm_rejected"] > 0
    b, _ = orc.rhs(g, f)
    assert np.linalg.norm(b - orc.apply(g, x[0])) / np.linalg.norm(b) <= 1e-7 * 1.001
    # every iteration is a CG step or a (rejected) line-search step; blocks
    # have at most 3 CG steps (a convergence check can end the last one early)
    assert s0["iters_cg"] + s0["dlsm_rejected"] == s0["iters_total"]
    full, rem = divmod(s0["iters_total"], 5)
    assert 3 * full <= s0["iters_cg"] <= 3 * full + min(rem, 3)


def _net(ppe, cfg, seed):
    p = onet.round_bf16_params(cfg, onet.init_params(cfg, np.random.default_rng(seed)))
    gcfg = ppe.ppe_net_config_default(levels=cfg.levels, base_channels=cfg.base_channels)
    net = ppe.Net(gcfg, seed=0)
    ppe.ppe_net_set_params(net, onet.flatten(cfg, p))
    return net, p


def test_network_round_matches_oracle(ppe, orc):
    cfg = onet.NetConfig(levels=3, base_channels=16)
    g = inputs.with_ellipse(inputs.make_grid(64, 48, 2.0, 1.5), np.random.default_rng(1))
    net, p = _net(ppe, cfg, 21)
    prob = ppe.ppe_problem_create(g)
    f = inputs.grf(g, 2).astype(np.float32)
    b, _ = orc.rhs(g, f)
    prov = onet.provider(p, cfg, g, g.mask)
    for k in (4, 5):
        st, stats, x = _solve(ppe, prob, net, f, tol=0.0, max_iter=k)
        xo, so, _ = orc.hybrid(g, b, prov, tol=0.0, max_iter=k, num_cg=3, num_dlsm=2)
        xo = orc.remove_mean(xo)
        assert stats[0]["iters_total"] == k
        assert np.linalg.norm(x[0] - xo) / np.linalg.norm(xo) <= 5e-2


def test_network_hybrid_converges(ppe, orc):
    cfg = onet.NetConfig(levels=3, base_channels=16)
    g = inputs.with_ellipse(inputs.make_grid(64, 64, 1.5), np.random.default_rng(2))
    net, p = _net(ppe, cfg, 22)
    prob = ppe.ppe_problem_create(g)
    f = inputs.gaussian_bumps(g, 6).astype(np.float32)
    b, _ = orc.rhs(g, f)
    st, stats, x = _solve(ppe, prob, net, f, tol=1e-8, max_iter=50000)
    assert st == ppe.PPE_OK
    s0 = stats[0]
    assert np.linalg.norm(b - orc.apply(g, x[0])) / np.linalg.norm(b) <= 1e-8 * 1.001
    xs = direct.separable_solve(g, b)
    assert np.linalg.norm(x[0] - xs) / np.linalg.norm(xs) <= 1e-6
    assert s0["iters_dlsm"] + s0["dlsm_rejected"] + s0["iters_cg"] == s0["iters_total"]


def test_batched_hybrid_equals_single(ppe, orc):
    cfg = onet.NetConfig(levels=3, base_channels=16)
    g = inputs.make_grid(48, 48, 2.0)
    net, p = _net(ppe, cfg, 23)
    prob = ppe.ppe_problem_create(g)
    fs = np.stack([inputs.grf(g, s) for s in range(3)]).astype(np.float32)
    st, stats, x = _solve(ppe, prob, net, fs, tol=1e-6, max_iter=20000)
    for s in range(3):
        st1, stats1, x1 = _solve(ppe, prob, net, fs[s], tol=1e-6, max_iter=20000)
        assert stats1[0]["iters_total"] == stats[s]["iters_total"]
        np.testing.assert_allclose(x1[0], x[s], rtol=0, atol=1e-12 * np.abs(x[s]).max())


def test_hybrid_argument_checks(ppe):
    g = inputs.make_grid(60, 64, 1.0)
    prob = ppe.ppe_problem_create(g)
    f = torch.zeros((1, 64, 60), dtype=torch.float32, device="cuda")
    x = torch.zeros((1, 64, 60), dtype=torch.float64, device="cuda")
    net = ppe.Net(ppe.ppe_net_config_default(), seed=0)
    with pytest.raises(ppe.PPEError) as ei:
        ppe.ppe_solve_hybrid(prob, net, f, x)
    assert ei.value.status == ppe.PPE_ERR_SHAPE
    with pytest.raises(ppe.PPEError):
        ppe.ppe_solve_hybrid(prob, None, f, x)
    with pytest.raises(ppe.PPEError):
        ppe.ppe_solve_hybrid(prob, None, f, x, ppe.ppe_solve_opts_default(direction=9))
