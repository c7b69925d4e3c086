"""Consecutive pressure solves on one grid, as a time-stepping flow solver makes
them (Sec. 2.5: the matrix and the preconditioner are built once, at the first
time step, and reused by every later one; Sec. 3 times the PPE over 20 000
consecutive time steps).

The sources come from the caller (`inputs.travelling_grf` makes a synthetic
sequence). Each step is one call of the library's solve on the device-resident
source of that step. With `warm` the solution of the previous step is the
initial guess of the next one (the paper does not state its initial guess; a
cold start from zero is the default). Every solve runs in the library's
kernels; this module only orders the calls and collects their statistics.
"""
import time


def run(ppe, prob, fs, x, opts, net=None, warm=False):
    """Solve fs[t] for t = 0, 1, ... in order.

    ppe   -- the loaded binding module
    prob  -- the grid's problem handle, created once for the whole sequence
    fs    -- device float32 tensor [steps, ny, nx] of sources
    x     -- device float64 tensor [1, ny, nx]; holds the last step's solution
             on return (and the first initial guess when warm)
    opts  -- solve options; zero_x0 is taken from `warm` per step
    net   -- a network for the hybrid solve, or None for plain PCG

    Returns (ms_total, per-step stats list, statuses). The time is wall-clock
    over the whole sequence, with the device synchronised before and after.
    """
    import torch
    opts.zero_x0 = 0 if warm else 1
    stats, status = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(fs.shape[0]):
        f = fs[t:t + 1]
        if net is None:
            st, s = ppe.ppe_solve_plain(prob, f, x, opts)
        else:
            st, s = ppe.ppe_solve_hybrid(prob, net, f, x, opts)
        status.append(st)
        stats.append(s[0])
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3, stats, status


def summary(ms, stats, status, ok):
    """Totals of one run: time, iterations per step, and convergence."""
    it = [s["iters_total"] for s in stats]
    n = len(it)
    return {"steps": n, "ms_total": ms, "ms_per_step": ms / max(n, 1),
            "iters_mean": sum(it) / max(n, 1), "iters_min": min(it, default=0), "iters_max": max(it, default=0),
            "iters_first": it[0] if it else 0, "iters_last": it[-1] if it else 0,
            "converged": sum(1 for st in status if st == ok),
            "max_rel_res_true": max((s["rel_res_true"] for s in stats), default=0.0)}
