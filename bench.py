#!/usr/bin/env python3
"""Benchmark of the pressure Poisson solve on one MI355X.

Workload (seeded, synthetic): a 1024 x 1024 cell-centred grid on the unit
square, tanh-stretched in x and y with beta = 1.75 (max/min spacing 8.8),
an elliptical obstacle mask (centre U[0.2, 0.8]^2, semi-axes U[0.05, 0.15],
angle U[0, pi)), and a Gaussian-random-field source (squared-exponential
covariance, length 0.05, 512 random Fourier features). Each step solves the
system from x0 = 0 to relative residual 1e-6 (FP64 true residual) with
Jacobi-PCG; `value` is that plain solve's rate.

Beside it the line always carries the hybrid half of the comparison
(config["hybrid"]): the same system solved by the hybrid PCG + line-search
method of Sec. 2.2 (Num_CG = 3, Num_DLSM = 2) with the network saved at
--hybrid PATH, or, without one, with the default network at its seeded
random initialisation (the control), each run capped at --hybrid-max-iter
iterations and reported as converged or not, with the device time split
into CG-type, network and line-search parts. config["hybrid_trained"]
repeats it with a network the run trains itself (the default network,
trained at 64^2 on Lanczos-Ritz vectors, about a minute), and compares
hybrid with plain PCG on held-out 64^2 systems, where that network was
trained. config["mgpcg"] and
config["hybrid_mgpcg"] repeat both with the multigrid-preconditioned CG
(the paper's strongest CG-type, MGPCG-4), and config["icpcg"] and
config["hybrid_icpcg"] with incomplete-Cholesky PCG (IC(0) in red-black
ordering, the paper's main comparison CG-type).

`roofline` reports the dominant kernel (the launch of the PCG form that
runs) on the algorithmic basis of 32 bytes per cell and PCG iteration (the
two-phase iteration's reads and writes of HBM-resident FP32 vectors), times
the iterations one launch makes, over its average launch duration (HIP
events attached to the launches); the kernel's own bytes per launch are
given beside it. config["hbm_resident_batch"] repeats the solve for 32
right-hand sides on the same grid, whose 1.1 GB of state cannot stay in the
256 MB last-level cache. config["mixed_batch"] solves one system on each
of 48 grids of uneven sizes (128 to 1024 cells per axis): plain PCG in one
work list, the hybrid in lock step with the network forwards of all grids
grouped into one launch per layer, and that grouped forward timed against
one forward per grid. `cpu_baseline` times the FP64 oracle on a bounded
sample (a fixed number of PCG iterations on the same system, scaled to the
iteration count of a full solve).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "PPE solves/sec to rel-res 1e-6, hybrid vs plain PCG, 1024² grid; HBM GB/s"
HBM_PEAK_GBS = 8000.0
BYTES_ITER = 32     # algorithmic basis per cell and PCG iteration (two-phase reads and writes)
BYTES_PCG1 = 24     # own bytes per cell: reads r, p, x_c; writes r, p, x_c (FP32)
BYTES_PCG2 = 24     # own bytes per cell and launch of two iterations: the same six FP32 vectors
BYTES_PHASE_A = 20  # own bytes per cell: reads r, p_old, x_c; writes p, x_c (FP32)
BYTES_PHASE_B = 12  # own bytes per cell: reads p, r; writes r (FP32)
HBM_BATCH = 32      # right-hand sides of the HBM-resident batch
MIXED_N = 48        # grids of the mixed-size batch
MIXED_ITERS = 60    # iterations of its hybrid solves


def workload(n=1024, beta=1.75, seed=0):
    from paper_2604_01800_amd import inputs
    g = inputs.with_ellipse(inputs.make_grid(n, n, beta), np.random.default_rng(seed))
    f = inputs.grf(g, seed).astype(np.float32)
    return g, f


def measured_traffic(kernel, record):
    """HBM bytes per launch from a committed hardware-counter run, if the
    kernel sources are unchanged since then (else None)."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", record)
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for f in rec["kernel_sources"]:
            h.update(open(os.path.join(here, f), "rb").read())
        if h.hexdigest() != rec["sources_sha256"]:
            return None
        return float(rec["traffic_bytes_per_launch"][kernel])
    except (OSError, KeyError, ValueError):
        return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, f, iters_full, sample_iters):
    """Single-threaded FP64 oracle PCG: time `sample_iters` iterations, scale."""
    import oracle
    b, _ = oracle.rhs(g, f)
    t0 = time.perf_counter()
    oracle.pcg(g, b, tol=0.0, max_iter=sample_iters)
    dt = time.perf_counter() - t0
    per_iter = dt / sample_iters
    return {
        "value": 1.0 / (per_iter * iters_full),
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{sample_iters} FP64 Jacobi-PCG iterations of the C oracle on the same {g.nx}x{g.ny} "
                  f"system ({dt:.1f} s, {per_iter * 1e3:.2f} ms/iteration), scaled to the {iters_full} "
                  f"iterations of a full solve to 1e-6",
        "cpu_model": cpu_model(),
        "host_threads_visible": os.cpu_count(),
    }


def hybrid_run(ppe, torch, prob, f, x, args, net=None, name=None):
    """Hybrid solves (Num_CG = 3, Num_DLSM = 2) of the same system, timed like
    the plain solve (one warm-up, then args.steps, capped at 2 since a hybrid
    solve can take seconds). The network is `net` (described by `name`), else
    the one saved at args.hybrid, else the default network at its seeded
    random initialisation."""
    if net is None:
        net = ppe.Net(ppe.ppe_net_config_default(), seed=0)
        if args.hybrid:
            ppe.ppe_net_load(net, args.hybrid)
            name = os.path.basename(args.hybrid)
        else:
            name = "default network (4 levels, 32-256 channels), seeded random initialisation (control)"
    o = ppe.ppe_solve_opts_default(tol=args.tol, zero_x0=1, max_iter=args.hybrid_max_iter)
    # the forward's tile widths tuned on this grid, as the plain solve's launch configuration is
    tiles = ppe.ppe_tune_net(net, prob, nb=1, reps=10)
    ppe.ppe_solve_hybrid(prob, net, f, x, o)
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 2))
    t0 = time.perf_counter()
    for _ in range(steps):
        st, stats = ppe.ppe_solve_hybrid(prob, net, f, x, o)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    s0 = stats[0]
    out = {"network": name, "converged": st == ppe.PPE_OK,
           "status": "converged" if st == ppe.PPE_OK else f"not converged within {args.hybrid_max_iter} iterations",
           "ms_per_solve": ms, "solves_per_s": 1e3 / ms if st == ppe.PPE_OK else 0.0,
           "iters": s0["iters_total"], "iters_cg": s0["iters_cg"], "iters_dlsm": s0["iters_dlsm"],
           "dlsm_rejected": s0["dlsm_rejected"], "rel_res_true": s0["rel_res_true"],
           "max_iter": args.hybrid_max_iter, "num_cg": 3, "num_dlsm": 2,
           "ms_pcg": s0["ms_pcg"], "ms_net": s0["ms_net"], "ms_dlsm": s0["ms_dlsm"],
           "net_tiles_tuned": {"32": sum(t == 32 for t, _, _ in tiles.values()),
                               "64": sum(t == 64 for t, _, _ in tiles.values())}}
    return out


def trained_run(ppe, torch, prob, f, x, args):
    """The hybrid half with a network trained here: the default network
    trained by the library at 64^2 (Eq. 19 loss, Adam with cosine decay from
    5e-4, batch 16, args.train_steps steps) on Lanczos-Ritz training vectors
    (Eqs. 14-16: 512 vectors from Lanczos bases of m = 0.14 N on 16 random
    stretched grids, b = 0.6). Reported: the hybrid solve of the benchmark
    system with it (timed like the plain solve), and hybrid against plain
    Jacobi-PCG on six held-out 64^2 systems (random stretching and ellipse,
    GRF sources), iterations and device ms each."""
    from paper_2604_01800_amd import training
    t0 = time.perf_counter()
    n = 64
    grids, R = training.make_ritz_pool(n, 512, seed=1, grids=16)
    probs = [ppe.ppe_problem_create(g) for g in grids]
    net = ppe.Net(ppe.ppe_net_config_default(), seed=7)
    losses = training.train(net, grids, R, steps=args.train_steps, batch=16, lr=5e-4, problems=probs,
                            schedule="cosine")
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    recipe = (f"default network trained here at 64^2: {args.train_steps} Adam steps (Eq. 19 loss, cosine decay from "
              f"5e-4, batch 16) on 512 Lanczos-Ritz vectors from 16 grids")
    out = {"training": {"recipe": recipe, "seconds": round(train_s, 1),
                        "loss_first_50": float(np.mean(losses[:50])), "loss_last_200": float(np.mean(losses[-200:]))},
           "benchmark_system": hybrid_run(ppe, torch, prob, f, x, args, net=net, name=recipe)}
    rows = training.evaluate(net, n, count=6, max_iter=args.hybrid_max_iter)
    ratio = [r["hybrid_iters"] / r["plain_iters"] for r in rows]
    out["held_out_64"] = {
        "systems": len(rows),
        "plain_iters": [r["plain_iters"] for r in rows],
        "hybrid_iters": [r["hybrid_iters"] for r in rows],
        "hybrid_dlsm": [r["hybrid_dlsm"] for r in rows],
        "hybrid_converged": [r["hybrid_converged"] for r in rows],
        "plain_ms": [round(r["plain_ms"], 3) for r in rows],
        "hybrid_ms": [round(r["hybrid_ms"], 3) for r in rows],
        "median_iter_ratio_hybrid_over_plain": float(np.median(ratio)),
        "median_ms_ratio_hybrid_over_plain": float(np.median([r["hybrid_ms"] / r["plain_ms"] for r in rows])),
    }
    return out


def mg_run(ppe, torch, prob, f, x, args):
    """Multigrid-preconditioned CG (the paper's MGPCG-4 CG-type) on the same
    system, and the hybrid over it (the network of the hybrid leg), timed
    like the plain solve."""
    out = {}
    o = ppe.ppe_solve_opts_default(tol=args.tol, zero_x0=1, precond=ppe.PPE_PC_MG, mg_levels=4,
                                   reliable_delta=args.mg_delta)
    ppe.ppe_solve_plain(prob, f, x, o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st, stats = ppe.ppe_solve_plain(prob, f, x, o)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    s0 = stats[0]
    out["mgpcg"] = {"converged": st == ppe.PPE_OK, "ms_per_solve": ms, "solves_per_s": 1e3 / ms,
                    "iters": s0["iters_total"], "reliable_updates": s0["reliable_updates"],
                    "rel_res_true": s0["rel_res_true"], "levels": 4, "reliable_delta": args.mg_delta,
                    "smoother": "Chebyshev degree 2 on D^-1 A over [0.2, 2], pre and post",
                    "coarsest": "exact separable FP64 solve (128 x 128)"}
    net = ppe.Net(ppe.ppe_net_config_default(), seed=0)
    if args.hybrid:
        ppe.ppe_net_load(net, args.hybrid)
    oh = ppe.ppe_solve_opts_default(tol=args.tol, zero_x0=1, precond=ppe.PPE_PC_MG, mg_levels=4,
                                    reliable_delta=args.mg_delta, max_iter=args.mg_hybrid_max_iter)
    ppe.ppe_solve_hybrid(prob, net, f, x, oh)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, stats = ppe.ppe_solve_hybrid(prob, net, f, x, oh)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    s0 = stats[0]
    out["hybrid_mgpcg"] = {"network": os.path.basename(args.hybrid) if args.hybrid else "seeded random init (control)",
                           "converged": st == ppe.PPE_OK, "ms_per_solve": ms,
                           "solves_per_s": 1e3 / ms if st == ppe.PPE_OK else 0.0,
                           "iters": s0["iters_total"], "iters_cg": s0["iters_cg"], "iters_dlsm": s0["iters_dlsm"],
                           "rel_res_true": s0["rel_res_true"], "max_iter": args.mg_hybrid_max_iter,
                           "ms_pcg": s0["ms_pcg"], "ms_net": s0["ms_net"], "ms_dlsm": s0["ms_dlsm"]}
    return out


def ic_run(ppe, torch, prob, f, x, args):
    """Incomplete-Cholesky PCG (IC(0) in red-black ordering, the paper's
    ICPCG CG-type) on the same system, and the hybrid over it (the network of
    the hybrid leg), timed like the plain solve."""
    out = {}
    o = ppe.ppe_solve_opts_default(tol=args.tol, zero_x0=1, precond=ppe.PPE_PC_IC, max_iter=20000)
    ppe.ppe_solve_plain(prob, f, x, o)
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 3))
    t0 = time.perf_counter()
    for _ in range(steps):
        st, stats = ppe.ppe_solve_plain(prob, f, x, o)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    s0 = stats[0]
    out["icpcg"] = {"converged": st == ppe.PPE_OK, "ms_per_solve": ms, "solves_per_s": 1e3 / ms,
                    "iters": s0["iters_total"], "reliable_updates": s0["reliable_updates"],
                    "rel_res_true": s0["rel_res_true"],
                    "preconditioner": "IC(0) in red-black ordering (two passes over independent cells)"}
    net = ppe.Net(ppe.ppe_net_config_default(), seed=0)
    if args.hybrid:
        ppe.ppe_net_load(net, args.hybrid)
    oh = ppe.ppe_solve_opts_default(tol=args.tol, zero_x0=1, precond=ppe.PPE_PC_IC, max_iter=args.mg_hybrid_max_iter)
    t0 = time.perf_counter()
    st, stats = ppe.ppe_solve_hybrid(prob, net, f, x, oh)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    s0 = stats[0]
    out["hybrid_icpcg"] = {"network": os.path.basename(args.hybrid) if args.hybrid else "seeded random init (control)",
                           "converged": st == ppe.PPE_OK,
                           "status": "converged" if st == ppe.PPE_OK
                           else f"not converged within {args.mg_hybrid_max_iter} iterations",
                           "ms_per_solve": ms, "solves_per_s": 1e3 / ms if st == ppe.PPE_OK else 0.0,
                           "iters": s0["iters_total"], "iters_cg": s0["iters_cg"], "iters_dlsm": s0["iters_dlsm"],
                           "rel_res_true": s0["rel_res_true"], "max_iter": args.mg_hybrid_max_iter,
                           "ms_pcg": s0["ms_pcg"], "ms_net": s0["ms_net"], "ms_dlsm": s0["ms_dlsm"]}
    return out


def hbm_batch_run(ppe, torch, g, prob, args):
    """Plain solve of HBM_BATCH right-hand sides on the headline grid (state
    well beyond the last-level cache) and the average launch time of its PCG
    kernel; bandwidth on the 32 B/cell/iteration basis and on the kernel's
    own bytes."""
    from paper_2604_01800_amd import inputs
    nb = HBM_BATCH
    f = torch.from_numpy(np.stack([inputs.grf(g, 1000 + k).astype(np.float32) for k in range(nb)])).cuda()
    x = torch.zeros((nb, g.ny, g.nx), dtype=torch.float64, device="cuda")
    o = ppe.ppe_solve_opts_default(tol=args.tol, zero_x0=1)
    variant, rows = ppe.ppe_get_tuning(prob, nb)
    ppe.ppe_solve_plain(prob, f, x, o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, stats = ppe.ppe_solve_plain(prob, f, x, o)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    po = ppe.ppe_solve_opts_default(tol=args.tol, variant=variant, rows_per_wave=rows)
    ms_a, ms_b = ppe.ppe_profile_pcg(prob, f, torch.zeros_like(x), po, reps=max(20, args.profile_reps // 4))
    N = g.nx * g.ny * nb
    per_launch = 2 if variant == ppe.PPE_PCG_TWO_STEP else 1
    own = {ppe.PPE_PCG_TWO_STEP: BYTES_PCG2, ppe.PPE_PCG_SINGLE_REDUCTION: BYTES_PCG1}.get(variant, BYTES_ITER)
    t_launch = (ms_a + ms_b) * 1e-3
    alg = BYTES_ITER * per_launch * N / t_launch / 1e9
    own_gbs = own * N / t_launch / 1e9
    del f, x
    torch.cuda.empty_cache()
    return {"nb": nb, "grid": [g.nx, g.ny], "state_GB": N * 32 / 1e9,
            "converged": st == ppe.PPE_OK, "ms_per_batch_solve": ms, "solves_per_s": nb * 1e3 / ms,
            "iters_max": max(s["iters_total"] for s in stats), "iters_min": min(s["iters_total"] for s in stats),
            "pcg_form": {1: "single", 2: "two_phase", 3: "two_step"}[variant], "rows_per_wave": rows,
            "kernel_ms": ms_a + ms_b, "iters_per_launch": per_launch,
            "GBps_32B_basis": alg, "frac_32B_basis": alg / HBM_PEAK_GBS,
            "own_bytes_per_cell_launch": own, "GBps_own_bytes": own_gbs, "frac_own_bytes": own_gbs / HBM_PEAK_GBS}


def mixed_batch_run(ppe, torch, args):
    """MIXED_N grids of uneven sizes from 128 to 1024 cells per axis (tanh
    grids with random stretching, GRF sources): the plain solves to the
    tolerance in one work list, the hybrid solves in lock step for
    MIXED_ITERS iterations (random-init network), and the network forward on
    one field of every grid as one grouped launch per layer against one
    forward launch sequence per grid."""
    from paper_2604_01800_amd import inputs
    rng = np.random.default_rng(51)
    sizes = list(range(128, 1025, 64))
    shapes = [(int(rng.choice(sizes)), int(rng.choice(sizes))) for _ in range(MIXED_N)]
    grids = [inputs.random_stretched_grid(nx, ny, rng) for nx, ny in shapes]
    probs = [ppe.ppe_problem_create(gk) for gk in grids]
    fs = [torch.from_numpy(inputs.grf(gk, 500 + k).astype(np.float32)).cuda() for k, gk in enumerate(grids)]
    xs = [torch.zeros(f.shape, dtype=torch.float64, device="cuda") for f in fs]
    out = {"grids": MIXED_N, "cells": int(sum(nx * ny for nx, ny in shapes))}
    o = ppe.ppe_solve_opts_default(tol=args.tol)
    st, stats = ppe.ppe_solve_batch(probs, fs, xs, o)
    out["plain_converged"] = st == ppe.PPE_OK
    out["plain_ms"] = stats[0]["ms_total"]
    out["plain_solves_per_s"] = MIXED_N * 1e3 / stats[0]["ms_total"]
    net = ppe.Net(ppe.ppe_net_config_default(), seed=9)
    ho = ppe.ppe_solve_opts_default(tol=args.tol, max_iter=MIXED_ITERS)
    for rep in range(2):  # the first call also builds every grid's network constants
        for x in xs:
            x.zero_()
        st, hs = ppe.ppe_solve_batch(probs, fs, xs, ho, net=net)
    out["hybrid_iters"] = MIXED_ITERS
    out["hybrid_forwards_per_solve"] = hs[0]["iters_dlsm"]
    out["hybrid_ms"] = hs[0]["ms_total"]
    out["hybrid_ms_split"] = {"cg": hs[0]["ms_pcg"], "net": hs[0]["ms_net"], "dlsm": hs[0]["ms_dlsm"]}
    ys = [torch.empty_like(f) for f in fs]
    ppe.ppe_net_forward_batch(net, probs, fs, ys)
    reps = 5
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ppe.ppe_net_forward_batch(net, probs, fs, ys)
    torch.cuda.synchronize()
    out["forward_grouped_ms"] = (time.perf_counter() - t0) * 1e3 / reps
    for p, f, y in zip(probs, fs, ys):
        ppe.ppe_net_forward(net, p, f[None], y[None])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for p, f, y in zip(probs, fs, ys):
            ppe.ppe_net_forward(net, p, f[None], y[None])
    torch.cuda.synchronize()
    out["forward_per_grid_ms"] = (time.perf_counter() - t0) * 1e3 / reps
    del probs, fs, xs, ys
    torch.cuda.empty_cache()
    return out


def sequence_run(ppe, torch, g, prob, x, opts, form, rows, args):
    """Consecutive solves of a travelling source on one grid (the shape of the
    paper's 20 000-step PPE timings): plain PCG from x0 = 0 and warm-started,
    and the hybrid solve likewise when a network is given. Prints one JSON line."""
    from paper_2604_01800_amd import inputs, sequence
    fs = torch.from_numpy(inputs.travelling_grf(g, 0, args.sequence, shift=args.seq_shift)).cuda()
    runs = {"pcg_x0_zero": (None, False), "pcg_warm": (None, True)}
    if args.hybrid:
        net = ppe.Net(ppe.ppe_net_config_default(), seed=0)
        ppe.ppe_net_load(net, args.hybrid)
        runs.update({"hybrid_x0_zero": (net, False), "hybrid_warm": (net, True)})
    out = {}
    for name, (net, warm) in runs.items():
        o = ppe.ppe_solve_opts_default(tol=args.tol, variant=opts.variant, rows_per_wave=opts.rows_per_wave,
                                       max_iter=args.hybrid_max_iter if net is not None else opts.max_iter)
        x.zero_()
        sequence.run(ppe, prob, fs[:1], x, o, net=net, warm=False)  # warm-up (graphs, workspaces)
        x.zero_()
        ms, stats, status = sequence.run(ppe, prob, fs, x, o, net=net, warm=warm)
        out[name] = sequence.summary(ms, stats, status, ppe.PPE_OK)
    print(json.dumps({"sequence": out, "grid": [g.nx, g.ny], "shift_per_step": args.seq_shift,
                      "tol": args.tol, "pcg_form": form, "rows_per_wave": rows,
                      "workload": "travelling GRF source (l = 0.05) on the headline grid, one solve per step"}),
          flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--cpu-iters", type=int, default=2400)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-reps", type=int, default=200)
    ap.add_argument("--variant", choices=["auto", "single", "two_phase", "two_step"], default="auto",
                    help="PCG iteration form: tuned on the workload before timing (auto, default), "
                         "one reduction per iteration, or two")
    ap.add_argument("--rows", type=int, default=0, choices=[0, 2, 4, 8, 16, 20, 24],
                    help="tile height (rows per wavefront); 0 = tuned or default")
    ap.add_argument("--network-forward", type=int, default=0, metavar="K",
                    help="time K forwards of the default DeepONet (random weights) on the workload's grid "
                         "instead (for kernel traces of the network)")
    ap.add_argument("--tune-net", action="store_true",
                    help="with --network-forward: also time the forward after tile-width tuning")
    ap.add_argument("--train-step", type=int, default=0, metavar="K",
                    help="time K training steps (forward, backward, Adam) of the default DeepONet on a pool of "
                         "--train-batch fabricated n x n systems instead (use with --n 256)")
    ap.add_argument("--train-batch", type=int, default=64)
    ap.add_argument("--hybrid", default=None, metavar="PATH",
                    help="network for the hybrid leg, saved by ppe_net_save (default configuration); without it "
                         "the hybrid leg runs the default network at its seeded random initialisation")
    ap.add_argument("--hybrid-max-iter", type=int, default=3000)
    ap.add_argument("--train-steps", type=int, default=12000,
                    help="Adam steps of the network trained for config['hybrid_trained'] (0: skip that leg)")
    ap.add_argument("--no-hbm-batch", action="store_true", help="skip the HBM-resident batch leg")
    ap.add_argument("--no-mixed-batch", action="store_true", help="skip the mixed-size batch leg")
    ap.add_argument("--mg-delta", type=float, default=0.1,
                    help="reliable-update threshold of the multigrid legs")
    ap.add_argument("--mg-hybrid-max-iter", type=int, default=500)
    ap.add_argument("--sequence", type=int, default=0, metavar="T",
                    help="time T consecutive solves on the workload's grid instead, the source travelling "
                         "--seq-shift domain lengths per step (step 0 is the headline source), from x0 = 0 "
                         "and warm-started from the previous step; with --hybrid also the hybrid solve")
    ap.add_argument("--seq-shift", type=float, default=0.001)
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the phase-kernel timing launches and a 64 MiB calibration copy "
                         "(for hardware-counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2604_01800_amd import ppe

    ppe.lib()
    torch.cuda.set_device(0)
    if args.train_step:
        from paper_2604_01800_amd import training
        grids, probs, Rd = training.make_pool(args.n, args.train_batch, seed=3)
        net = ppe.Net(ppe.ppe_net_config_default(), seed=1)
        training.train(net, grids, Rd, steps=3, batch=args.train_batch, lr=1e-4, problems=probs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        training.train(net, grids, Rd, steps=args.train_step, batch=args.train_batch, lr=1e-4, problems=probs)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / args.train_step * 1e3
        print(json.dumps({"train_step_ms": ms, "grid": [args.n, args.n], "batch": args.train_batch,
                          "steps": args.train_step}), flush=True)
        return
    g, f_np = workload(args.n)
    prob = ppe.ppe_problem_create(g)
    f = torch.from_numpy(f_np[None]).cuda()
    x = torch.zeros((1, g.ny, g.nx), dtype=torch.float64, device="cuda")
    if args.network_forward:
        net = ppe.Net(ppe.ppe_net_config_default(), seed=1)
        r = torch.from_numpy(f_np[None]).cuda()
        y = torch.zeros_like(r)
        for _ in range(3):
            ppe.ppe_net_forward(net, prob, r, y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.network_forward):
            ppe.ppe_net_forward(net, prob, r, y)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / args.network_forward * 1e3
        line = {"network_forward_ms": ms, "grid": [g.nx, g.ny], "forwards": args.network_forward}
        if args.tune_net:  # the same after tile-width tuning on this grid
            tiles = ppe.ppe_tune_net(net, prob, nb=1, reps=20)
            for _ in range(3):
                ppe.ppe_net_forward(net, prob, r, y)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.network_forward):
                ppe.ppe_net_forward(net, prob, r, y)
            torch.cuda.synchronize()
            line["network_forward_tuned_ms"] = (time.perf_counter() - t0) / args.network_forward * 1e3
            line["tuned_tiles"] = {k: t for k, (t, _, _) in tiles.items()}
        print(json.dumps(line), flush=True)
        return

    variant = {"auto": ppe.PPE_PCG_AUTO, "single": ppe.PPE_PCG_SINGLE_REDUCTION,
               "two_phase": ppe.PPE_PCG_TWO_PHASE, "two_step": ppe.PPE_PCG_TWO_STEP}[args.variant]
    opts = ppe.ppe_solve_opts_default(tol=args.tol, zero_x0=1, variant=variant)
    tuning = None
    if variant == ppe.PPE_PCG_AUTO and not args.kernels_only and args.rows == 0:
        # Launch-configuration tuning on the workload itself, before any timing.
        tuning = ppe.ppe_tune_pcg(prob, f, torch.zeros_like(x), reps=50)
        variant, rows = tuning["variant"], tuning["rows_per_wave"]
    else:
        rows = args.rows or (ppe.ppe_get_tuning(prob, 1)[1] if variant == ppe.PPE_PCG_AUTO else 0)
        if variant == ppe.PPE_PCG_AUTO:
            variant = ppe.ppe_get_tuning(prob, 1)[0]
    opts = ppe.ppe_solve_opts_default(tol=args.tol, zero_x0=1, variant=variant, rows_per_wave=rows)
    form = {ppe.PPE_PCG_SINGLE_REDUCTION: "single", ppe.PPE_PCG_TWO_PHASE: "two_phase",
            ppe.PPE_PCG_TWO_STEP: "two_step"}[variant]

    if args.sequence:
        sequence_run(ppe, torch, g, prob, x, opts, form, rows, args)
        return

    if args.kernels_only:
        ms_a, ms_b = ppe.ppe_profile_pcg(prob, f, x, opts, reps=args.profile_reps)
        src = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        ms_c = ppe.ppe_profile_copy(src, dst, reps=args.profile_reps)
        torch.cuda.synchronize()
        print(json.dumps({"variant": args.variant, "kernel_ms": [ms_a, ms_b], "copy_64MiB_ms": ms_c}), flush=True)
        return

    for _ in range(args.warmup):
        ppe.ppe_solve_plain(prob, f, x, opts)
    torch.cuda.synchronize()
    stats_all = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st, stats = ppe.ppe_solve_plain(prob, f, x, opts)
        stats_all.append(stats[0])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / args.steps * 1e3
    s0 = stats_all[-1]
    if st != ppe.PPE_OK:
        print(f"solve did not converge: {s0}", file=sys.stderr)

    # Dominant kernel, timed with HIP events attached to its own launches.
    xt = torch.zeros_like(x)
    ms_a, ms_b = ppe.ppe_profile_pcg(prob, f, xt, opts, reps=args.profile_reps)
    N = g.nx * g.ny
    iters = s0["iters_total"]
    if form == "two_step":
        kname, own, per_launch = "k_pcg2 (two PCG iterations per launch)", BYTES_PCG2, 2
        record, tkey, t_launch = "pcg2_1024_plain.counters.json", "k_pcg2", ms_a
    elif form == "single":
        kname, own, per_launch = "k_pcg1 (single-reduction PCG iteration)", BYTES_PCG1, 1
        record, tkey, t_launch = "pcg1_1024_plain.counters.json", "k_pcg1", ms_a
    else:
        kname, own, per_launch = "k_pcg_a + k_pcg_b (the two phases of one PCG iteration)", BYTES_ITER, 1
        record, tkey, t_launch = "pcg_phases_1024_plain.counters.json", "k_pcg_a", ms_a + ms_b
    alg_bytes = BYTES_ITER * per_launch * N
    ach = alg_bytes / (t_launch * 1e-3) / 1e9
    own_gbs = own * N / (t_launch * 1e-3) / 1e9
    # Whole-solve rate on the same 32 B/cell/iteration basis.
    pcg_gbs = BYTES_ITER * N * iters / (ms_per_step * 1e-3) / 1e9

    out = {
        "metric": METRIC,
        "value": 1e3 / ms_per_step,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"plain Jacobi-PCG, {g.nx}x{g.ny} tanh grid beta 1.75, ellipse mask, GRF source "
                        f"l=0.05, x0=0, rel-res {args.tol:g} on the FP64 true residual",
            "pcg_form": form,
            "rows_per_wave": rows,
            "tuning_us_per_iter": None if tuning is None else
                {f"{k[0]}/R{k[1]}": round(v, 2) for k, v in tuning["us_per_iter"].items()},
            "iters": iters,
            "reliable_updates": s0["reliable_updates"],
            "rel_res_true": s0["rel_res_true"],
            "precision": "FP32 vectors, FP64 reductions and solution accumulator",
            "effective_pcg_GBps_32B_basis": pcg_gbs,
            "kernel_ms": [ms_a, ms_b],
        },
        "roofline": {
            "kernel": kname,
            "bound": "hbm",
            "achieved": ach,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS,
            "traffic": measured_traffic(tkey, record),
            "basis": f"{BYTES_ITER} B/cell per PCG iteration x {per_launch} iteration(s) per launch x {N} cells",
            "algorithmic_bytes": alg_bytes,
            "kernel_ms": t_launch,
            "own_bytes": own * N,
            "own_GBps": own_gbs,
            "own_frac": own_gbs / HBM_PEAK_GBS,
        },
    }
    out["config"]["hybrid"] = hybrid_run(ppe, torch, prob, f, x, args)
    if args.train_steps > 0 and not args.hybrid:
        out["config"]["hybrid_trained"] = trained_run(ppe, torch, prob, f, x, args)
    out["config"].update(mg_run(ppe, torch, prob, f, x, args))
    out["config"].update(ic_run(ppe, torch, prob, f, x, args))
    if not args.no_hbm_batch:
        out["config"]["hbm_resident_batch"] = hbm_batch_run(ppe, torch, g, prob, args)
    if not args.no_mixed_batch:
        out["config"]["mixed_batch"] = mixed_batch_run(ppe, torch, args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, f_np, iters, args.cpu_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
