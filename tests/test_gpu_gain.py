"""What the trained network gains (Sec. 2.2-2.4): a DeepONet trained by the
library (Eq. 19 loss, Adam with cosine decay) on the paper's Lanczos-Ritz
training vectors (Eqs. 14-16: 512 vectors from Lanczos bases of m = 0.14 N
on 16 random stretched 64 x 64 grids, b = 0.6), against the same network
untrained and against plain PCG, on held-out systems with GRF sources.

Measured per held-out system:
  * the share of the A-norm error that one line search along NN(r) removes,
    (r.y)^2 / ((y.Ay)(r.A^+ r)), for the residual after 20 PCG iterations
    (A^+ r from a PCG solve to 1e-10);
  * iterations of the hybrid solve to 1e-6 (3 CG + 2 line-search steps per
    round) with the trained and with the untrained network;
  * iterations of plain PCG.
Training here is 12 000 Adam steps at lr 5e-4 (under a minute) and is
deterministic; six held-out systems. The line-search shares are the robust
signal (measured on MI355X: 0.27-0.81 trained against 1e-7-3e-3 untrained).
The hybrid's iteration count moves more: a rounding-level change in the
network output once moved the trained/plain ratios of the first four of
these systems from a median of 0.53 to 0.81, with the same weights, and the
median over four systems after 8 000 steps was 0.77. With 12 000 steps the
six ratios measured 0.23-2.1, median 0.40, which the bar of 0.7 leaves room
for. The bars: the hybrid solve with the trained network converges on every
system, its direction removes at least 10 % of the error and 100x the
untrained share, the median share is at least 30 %, the hybrid needs at most
half the untrained network's iterations (an unconverged solve counts as the
iteration limit), and on the median system it needs at most 0.7 times plain
PCG's iterations. The table printed by the test records the numbers."""
import numpy as np
import pytest
import torch

from paper_2604_01800_amd import inputs, training

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ppe():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_01800_amd import ppe as P
    P.lib()
    return P


def line_search_share(ppe, prob, area, net, r):
    """Share of the A-norm error of r removed by the exact line search along NN(r)."""
    e = torch.zeros_like(r)
    ppe.ppe_solve_plain(prob, (r / area).float(), e, ppe.ppe_solve_opts_default(tol=1e-10, zero_x0=1,
                                                                                max_iter=50000))
    rAr = float((r * e).sum())
    y = torch.zeros_like(r, dtype=torch.float32)
    ppe.ppe_net_forward(net, prob, r.float(), y)
    y = y.double()
    Ay = torch.zeros_like(y)
    ppe.ppe_apply_f64(prob, y, Ay)
    num, den = float((r * y).sum()), float((y * Ay).sum())
    return num * num / (den * rAr)


def test_trained_network_gain(ppe):
    n = 64
    grids, R = training.make_ritz_pool(n, 512, seed=1, grids=16)
    probs = [ppe.ppe_problem_create(g) for g in grids]
    cfg = ppe.ppe_net_config_default()
    trained = ppe.Net(cfg, seed=7)
    untrained = ppe.Net(cfg, seed=7)
    losses = training.train(trained, grids, R, steps=12000, batch=16, lr=5e-4, problems=probs, schedule="cosine")
    assert np.mean(losses[-200:]) < 0.25 * np.mean(losses[:50]), (np.mean(losses[:50]), np.mean(losses[-200:]))

    rng = np.random.default_rng(12345)
    rows = []
    max_iter = 20000
    for k in range(6):
        g = inputs.with_ellipse(inputs.random_stretched_grid(n, n, rng), rng)
        prob = ppe.ppe_problem_create(g)
        area = torch.from_numpy(np.outer(g.hy, g.hx)[None]).cuda()
        f_np = inputs.grf(g, 900 + k)
        f = torch.from_numpy(f_np.astype(np.float32)[None]).cuda()
        x = torch.zeros((1, n, n), dtype=torch.float64, device="cuda")
        o = ppe.ppe_solve_opts_default(tol=1e-6, zero_x0=1, max_iter=max_iter)
        st, sp = ppe.ppe_solve_plain(prob, f, x, o)
        assert st == ppe.PPE_OK
        row = {"plain": sp[0]["iters_total"]}
        for name, net in (("trained", trained), ("untrained", untrained)):
            st, sh = ppe.ppe_solve_hybrid(prob, net, f, x, o)
            row[name] = sh[0]["iters_total"] if st == ppe.PPE_OK else None
        # residual after 20 PCG iterations, in FP64
        ppe.ppe_solve_plain(prob, f, x, ppe.ppe_solve_opts_default(tol=0.0, zero_x0=1, max_iter=20))
        b = area * torch.from_numpy(f_np.astype(np.float32).astype(np.float64)[None]).cuda()
        b -= b.mean()
        Ax = torch.zeros_like(x)
        ppe.ppe_apply_f64(prob, x, Ax)
        r = b - Ax
        row["share_trained"] = line_search_share(ppe, prob, area, trained, r)
        row["share_untrained"] = line_search_share(ppe, prob, area, untrained, r)
        rows.append(row)
    for r in rows:
        print("held-out 64x64: plain %(plain)d it, hybrid trained %(trained)s it, untrained %(untrained)s it; "
              "line-search share trained %(share_trained).4f untrained %(share_untrained).2e" % r)
    for r in rows:
        assert r["trained"] is not None, r
        assert r["share_trained"] >= 0.1 and r["share_trained"] >= 100 * r["share_untrained"], r
    assert np.median([r["share_trained"] for r in rows]) >= 0.3, rows
    it_trained = sum(r["trained"] for r in rows)
    it_untrained = sum(max_iter if r["untrained"] is None else r["untrained"] for r in rows)
    assert 2 * it_trained <= it_untrained, (it_trained, it_untrained)
    assert np.median([r["trained"] / r["plain"] for r in rows]) <= 0.7, rows
