"""Self-training of the DeepONet on fabricated systems (Sec. 2.3-2.4 analogue).

The paper trains on a fixed set of fabricated right-hand sides built from
Lanczos-Ritz vectors of M, with the low end of the spectrum weighted up
(Eqs. 14-16). Here the fabricated set is a fixed pool of systems on random
stretched grids (tanh factors U[1, 2.5] per axis, an elliptical obstacle
mask each) whose right-hand sides are Gaussian random fields with the length
scale drawn log-uniformly in [0.05, 0.5] (longer scales weight the low end
of the spectrum), multiplied by the cell areas, projected to zero mean and
scaled to unit RMS. Training cycles through the pool in consecutive batches
and calls ppe_net_train_step (the residual loss of Eq. 19, Adam), with a
constant or cosine-decayed learning rate.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import inputs, ppe


def make_pool(n: int, count: int, seed: int = 0, ell_lo: float = 0.05, ell_hi: float = 0.5):
    """Returns (grids, R [count, n, n] float32)."""
    rng = np.random.default_rng(seed)
    grids, R = [], []
    for k in range(count):
        g = inputs.with_ellipse(inputs.random_stretched_grid(n, n, rng), rng)
        ell = float(np.exp(rng.uniform(np.log(ell_lo), np.log(ell_hi))))
        r = inputs.grf(g, int(rng.integers(1 << 31)), ell=ell) * np.outer(g.hy, g.hx)
        r -= r.mean()
        r /= np.sqrt(np.mean(r * r))
        grids.append(g)
        R.append(r.astype(np.float32))
    return grids, np.stack(R)


def cosine_lr(lr: float, step: int, steps: int) -> float:
    """Cosine decay of the learning rate from lr to 0 over `steps` (Sec. 2.4)."""
    return 0.5 * lr * (1.0 + math.cos(math.pi * step / steps))


def train(net, grids, R_dev, steps: int, batch: int, lr: float = 1e-3, log_every: int = 0, problems=None,
          schedule: str = "constant"):
    """Adam steps over consecutive batches of the pool (learning rate constant
    or cosine-decayed); returns the loss history."""
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
        opts = ppe.ppe_train_opts_default(lr=lr_k)
        loss, _ = ppe.ppe_net_train_step(net, probs[b0:b0 + batch], R_dev[b0:b0 + batch], opts)
        losses.append(loss)
        if log_every and (k + 1) % log_every == 0:
            print(f"train step {k + 1}/{steps} loss {np.mean(losses[-log_every:]):.4e} "
                  f"({time.perf_counter() - t0:.1f} s)", flush=True)
    return losses
