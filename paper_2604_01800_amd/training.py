"""Self-training of the DeepONet on fabricated systems (Sec. 2.3-2.4 analogue).

The paper trains on a fixed set of fabricated right-hand sides built from
Lanczos-Ritz vectors of M, with the low end of the spectrum weighted up
(Eqs. 14-16). Here the fabricated set is a fixed pool of systems on random
stretched grids (tanh factors U[1, 2.5] per axis, an elliptical obstacle
mask each) whose right-hand sides are Gaussian random fields with the length
scale drawn log-uniformly in [0.05, 0.5] (longer scales weight the low end
of the spectrum), multiplied by the cell areas, projected to zero mean and
scaled to unit RMS, or the Lanczos-Ritz vectors of Eqs. 14-16. Training
cycles through the pool in consecutive batches and calls ppe_net_train_step
(the residual loss of Eq. 19, or the supervised loss against the pool's FP64
solutions; Adam, optionally SAM), with a constant or cosine-decayed learning
rate.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import inputs, ppe


def make_pool(n: int, count: int, seed: int = 0, ell_lo: float = 0.05, ell_hi: float = 0.5):
    """count random stretched n x n grids (ellipse masks) with their sources
    drawn on the device by the library's generator (ppe_generate_rhs: random
    fields of log-uniform length scale in [ell_lo, ell_hi], times the cell
    area, zero mean, unit RMS). Returns (grids, problems, device R [count, n, n])."""
    import torch
    rng = np.random.default_rng(seed)
    grids = [inputs.with_ellipse(inputs.random_stretched_grid(n, n, rng), rng) for _ in range(count)]
    probs = [ppe.ppe_problem_create(g) for g in grids]
    R = torch.empty((count, n, n), dtype=torch.float32, device="cuda")
    ppe.ppe_generate_rhs(probs, ppe.ppe_train_opts_default(seed=seed, step=0, grf_len_lo=ell_lo, grf_len_hi=ell_hi),
                         R)
    return grids, probs, R


def generated_grids(n: int, count: int, seed: int = 0, step: int = 0):
    """count n x n grids drawn by the library's generator (ppe_generate_grid):
    tanh stretch factors in [1, 2.5] and an elliptic obstacle per sample."""
    return [ppe.ppe_generate_grid(n, n, seed, step, k) for k in range(count)]


def make_ritz_pool(n: int, count: int, seed: int = 0, grids: int = 16, m: int | None = None, b: float = 0.6,
                   log: bool = False):
    """Pool of Lanczos-Ritz training systems (Sec. 2.3, Eqs. 14-16): `grids`
    random stretched n x n grids (ellipse masks), a Lanczos basis of m vectors
    on each (default m = 0.14 N, the paper's m / N), and count / grids
    vectors drawn on each with weight 9 on the lowest b m Ritz vectors
    (log: one progress line per grid). Returns (grid list of length count,
    device R [count, n, n] float32)."""
    import torch
    if count % grids:
        raise ValueError("count must be a multiple of grids")
    rng = np.random.default_rng(seed)
    m = m or max(8, int(0.14 * n * n))
    per = count // grids
    R = torch.empty((count, n, n), dtype=torch.float32, device="cuda")
    gl = [None] * count
    t0 = time.perf_counter()
    # slot i * grids + k holds vector i of grid k, so consecutive batches mix
    # the grids; the vectors have unit RMS (L2 norm sqrt(N) instead of the 1
    # of Eq. 15), the scale of the other training data
    for k in range(grids):
        g = inputs.with_ellipse(inputs.random_stretched_grid(n, n, rng), rng)
        prob = ppe.ppe_problem_create(g)
        v0 = torch.from_numpy(rng.standard_normal((n, n))).cuda()
        r = ppe.Ritz(prob, m, v0)
        for i in range(per):
            slot = i * grids + k
            ppe.ppe_ritz_rhs(r, R[slot:slot + 1], seed=seed, step=k * per + i, b=b, scale=float(np.sqrt(n * n)))
            gl[slot] = g
        if log:
            print(f"ritz pool: grid {k + 1}/{grids} ({m} Lanczos steps, {time.perf_counter() - t0:.1f} s)", flush=True)
    return gl, R


def make_targets(probs, R, tol: float = 1e-10):
    """FP64 solutions e_s of A e_s = R_s (the targets of the supervised loss):
    each right-hand side turned into its source by the library
    (ppe_rhs_to_source) and solved with multigrid PCG where the grid allows
    it, else Jacobi-PCG. Returns a device float64 tensor shaped like R."""
    import torch
    n = R.shape[0]
    E = torch.zeros(R.shape, dtype=torch.float64, device="cuda")
    f = torch.empty_like(R[0:1])
    for k in range(n):
        p = probs[k]
        ppe.ppe_rhs_to_source(p, R[k:k + 1], f)
        mg = p.nx % 8 == 0 and p.ny % 8 == 0
        o = ppe.ppe_solve_opts_default(tol=tol, zero_x0=1, max_iter=200000,
                                       precond=ppe.PPE_PC_MG if mg else ppe.PPE_PC_JACOBI)
        st, _ = ppe.ppe_solve_plain(p, f, E[k:k + 1], o)
        if st != ppe.PPE_OK:
            raise RuntimeError(f"target solve {k} did not converge")
    return E


def cosine_lr(lr: float, step: int, steps: int) -> float:
    """Cosine decay of the learning rate from lr to 0 over `steps` (Sec. 2.4)."""
    return 0.5 * lr * (1.0 + math.cos(math.pi * step / steps))


def train(net, grids, R_dev, steps: int, batch: int, lr: float = 1e-3, log_every: int = 0, problems=None,
          schedule: str = "constant", clip_norm: float = 0.0, sam_rho: float = 0.0, data_seed: int = 0,
          targets=None, loss_kind: int = ppe.PPE_LOSS_SUPERVISED):
    """Adam steps over consecutive batches of the pool (learning rate constant
    or cosine-decayed; gradients clipped to clip_norm in L2 norm when it is
    positive; sharpness-aware with radius sam_rho when it is positive);
    returns the loss history. With R_dev None the sources of step k are drawn
    on the device by the library's generator (seed data_seed, step k). With
    targets (FP64 solutions of the pool's systems, make_targets) the loss is
    loss_kind against them (supervised or A-norm), else the residual loss of
    Eq. 19."""
    count = len(grids)
    if count % batch:
        raise ValueError("pool size must be a multiple of the batch")
    probs = problems or [ppe.ppe_problem_create(g) for g in grids]
    if schedule not in ("constant", "cosine"):
        raise ValueError(f"unknown schedule {schedule}")
    losses = []
    t0 = time.perf_counter()
    for k in range(steps):
        b0 = (k * batch) % count
        lr_k = cosine_lr(lr, k, steps) if schedule == "cosine" else lr
        opts = ppe.ppe_train_opts_default(lr=lr_k, clip_norm=clip_norm, sam_rho=sam_rho, seed=data_seed, step=k,
                                          loss_kind=ppe.PPE_LOSS_RESIDUAL if targets is None else loss_kind)
        # R_dev None: the library draws every batch's sources on the device
        R_k = None if R_dev is None else R_dev[b0:b0 + batch]
        T_k = None if targets is None else targets[b0:b0 + batch]
        loss, _ = ppe.ppe_net_train_step(net, probs[b0:b0 + batch], R_k, opts, target=T_k)
        losses.append(loss)
        if log_every and (k + 1) % log_every == 0:
            print(f"train step {k + 1}/{steps} loss {np.mean(losses[-log_every:]):.4e} "
                  f"({time.perf_counter() - t0:.1f} s)", flush=True)
    return losses


def evaluate(net, n, count=6, seed=12345, tol=1e-6, max_iter=20000, num_cg=3, num_dlsm=2):
    """Hybrid (with net; num_cg PCG iterations and num_dlsm line-search steps
    per round, Sec. 2.2) against plain Jacobi-PCG on held-out n x n systems
    (random stretching and ellipse, GRF source); returns one dict per system."""
    import torch
    rng = np.random.default_rng(seed)
    rows = []
    for k in range(count):
        g = inputs.with_ellipse(inputs.random_stretched_grid(n, n, rng), rng)
        prob = ppe.ppe_problem_create(g)
        f = torch.from_numpy(inputs.grf(g, 900 + k).astype(np.float32)[None]).cuda()
        x = torch.zeros((1, n, n), dtype=torch.float64, device="cuda")
        o = ppe.ppe_solve_opts_default(tol=tol, zero_x0=1, max_iter=max_iter, num_cg=num_cg, num_dlsm=num_dlsm)
        st_p, sp = ppe.ppe_solve_plain(prob, f, x, o)
        st_h, sh = ppe.ppe_solve_hybrid(prob, net, f, x, o)
        rows.append({"n": n, "system": k, "num_cg": num_cg, "num_dlsm": num_dlsm,
                     "plain_iters": sp[0]["iters_total"], "plain_ms": sp[0]["ms_device"],
                     "hybrid_iters": sh[0]["iters_total"], "hybrid_dlsm": sh[0]["iters_dlsm"],
                     "hybrid_ms": sh[0]["ms_device"], "hybrid_converged": st_h == ppe.PPE_OK})
    return rows


def main(argv=None):
    """Train a DeepONet on fabricated n x n systems and compare the hybrid
    solve with plain PCG on held-out systems (one JSON line per system)."""
    import argparse
    import json

    import torch
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--pool", type=int, default=2048)
    ap.add_argument("--steps", type=int, default=120000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--clip", type=float, default=0.0, help="global gradient-norm clip (0: none)")
    ap.add_argument("--sam", type=float, default=0.0, help="sharpness-aware radius (0: plain Adam)")
    ap.add_argument("--levels", type=int, default=0, help="U-Net levels (0: the library default, 4)")
    ap.add_argument("--base-channels", type=int, default=0,
                    help="channels of the finest level, doubling per level (0: the library default, 32); "
                         "the paper's network is --levels 5 --base-channels 40")
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--out", default=None, help="save the trained network here")
    ap.add_argument("--load", default=None, help="load this network instead of training one")
    ap.add_argument("--data", choices=["grf", "ritz", "generated"], default="grf",
                    help="training systems: Gaussian random fields, Lanczos-Ritz vectors (Eqs. 14-16), or "
                         "grids from the library's generator with sources drawn on the device at every step")
    ap.add_argument("--ritz-m", type=int, default=0,
                    help="Lanczos steps per grid of the Ritz pool (0: the paper's ratio, 0.14 N)")
    ap.add_argument("--ritz-grids", type=int, default=16, help="grids of the Ritz pool")
    ap.add_argument("--loss", choices=["residual", "supervised", "anorm"], default="residual",
                    help="the residual loss of Eq. 19, or the supervised or A-norm (line-search share) loss "
                         "against FP64 solutions of the pool")
    ap.add_argument("--eval-sizes", default="64,128,256")
    ap.add_argument("--eval-count", type=int, default=6, help="held-out systems at the training size")
    ap.add_argument("--sweep", action="store_true",
                    help="also sweep Num_CG and Num_DLSM over 1..5 on held-out n x n systems (Appendix A)")
    args = ap.parse_args(argv)
    ppe.lib()
    kw = {}
    if args.levels:
        kw["levels"] = args.levels
    if args.base_channels:
        kw["base_channels"] = args.base_channels
    net = ppe.Net(ppe.ppe_net_config_default(**kw), seed=args.seed)
    if args.load:
        ppe.ppe_net_load(net, args.load)
    else:
        if args.data == "ritz":
            grids, Rd = make_ritz_pool(args.n, args.pool, seed=1, grids=args.ritz_grids, m=args.ritz_m or None,
                                       log=True)
        elif args.data == "generated":
            grids, Rd = generated_grids(args.n, args.pool, seed=1), None
        else:
            grids, _, Rd = make_pool(args.n, args.pool, seed=1)
        probs = [ppe.ppe_problem_create(g) for g in grids]
        targets = None
        if args.loss != "residual":
            if Rd is None:
                raise SystemExit(f"--loss {args.loss} needs a fixed pool (--data grf or ritz)")
            targets = make_targets(probs, Rd)
        train(net, grids, Rd, steps=args.steps, batch=args.batch, lr=args.lr,
              log_every=max(1, args.steps // 20), problems=probs, schedule="cosine", clip_norm=args.clip,
              sam_rho=args.sam, targets=targets,
              loss_kind=ppe.PPE_LOSS_ANORM if args.loss == "anorm" else ppe.PPE_LOSS_SUPERVISED)
    if args.out:
        ppe.ppe_net_save(net, args.out)
    for n in (int(v) for v in args.eval_sizes.split(",") if v):
        for row in evaluate(net, n, count=args.eval_count if n == args.n else 3):
            print(json.dumps(row), flush=True)
    if args.sweep:
        for num_cg in range(1, 6):
            for num_dlsm in range(1, 6):
                rows = evaluate(net, args.n, count=6, num_cg=num_cg, num_dlsm=num_dlsm)
                print(json.dumps({"sweep": True, "n": args.n, "num_cg": num_cg, "num_dlsm": num_dlsm,
                                  "plain_iters": [r["plain_iters"] for r in rows],
                                  "hybrid_iters": [r["hybrid_iters"] for r in rows],
                                  "hybrid_dlsm": [r["hybrid_dlsm"] for r in rows],
                                  "plain_ms": [round(r["plain_ms"], 3) for r in rows],
                                  "hybrid_ms": [round(r["hybrid_ms"], 3) for r in rows],
                                  "converged": [r["hybrid_converged"] for r in rows]}), flush=True)


if __name__ == "__main__":
    main()
