"""TEST INFRASTRUCTURE — the CPU oracle for the pressure Poisson solve.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package. The GPU library never imports, links or calls it, and it shares
no code with the GPU library. Everything here is FP64 and single-threaded:

* ``ppe_oracle.c`` (loaded through ctypes): the finite-volume operator of Eq. 10,
  its diagonal, the right-hand-side preparation, textbook Jacobi-PCG and the
  hybrid CG / line-search controller of Sec. 2.2 with a pluggable error provider.
* ``direct``: two independent direct solves used to pin the iterative ones.
* ``net``: the DeepONet branch/trunk network and Mesh-Conv layers (Sec. 2.4)
  in plain PyTorch CPU float64, the Eq. 19 loss, its autograd gradient, the
  sharpness-aware gradient and its own BF16 rounding of parameters.
* ``mg``: the multigrid V-cycle preconditioner (the paper's MGPCG-4 CG-type,
  Sec. 2.5), geometric on the tensor grid, for ``pcg``/``hybrid`` with
  ``precond = 2``.
* ``ic``: the incomplete-Cholesky preconditioner IC(0) in red-black
  ordering (the paper's ICPCG CG-type, Sec. 2.5), for ``precond = 2``.
* ``datagen`` and ``ritz``: the training-data generators (random-field
  sources, per-sample grids, and the Lanczos-Ritz vectors of Eqs. 14-16).

The package imports nothing from the GPU library's package; the tests feed
both sides from the seeded input module only.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ppe_oracle.c")
_LIB = os.path.join(_HERE, "libppe_oracle.so")


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, no fast-math, one thread)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("xc", ctypes.c_void_p), ("yc", ctypes.c_void_p),
                ("hx", ctypes.c_void_p), ("hy", ctypes.c_void_p),
                ("mask", ctypes.c_void_p), ("mask_mode", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("converged", ctypes.c_int32), ("iters_total", ctypes.c_int32),
                ("iters_cg", ctypes.c_int32), ("iters_dlsm", ctypes.c_int32),
                ("dlsm_rejected", ctypes.c_int32), ("breakdowns", ctypes.c_int32),
                ("res_final", ctypes.c_double)]


PROVIDER = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p,
                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double))

_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        _lib.orc_apply.argtypes = [ctypes.POINTER(_Grid), vp, vp]
        _lib.orc_diag.argtypes = [ctypes.POINTER(_Grid), vp]
        _lib.orc_dot.argtypes = [i64, vp, vp]
        _lib.orc_dot.restype = d
        _lib.orc_rhs.argtypes = [ctypes.POINTER(_Grid), vp, vp]
        _lib.orc_rhs.restype = d
        _lib.orc_hybrid.argtypes = [ctypes.POINTER(_Grid), vp, vp, ctypes.c_int, d, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, PROVIDER, vp,
                                    ctypes.POINTER(Stats), vp, i32]
        _lib.orc_hybrid_pc.argtypes = [ctypes.POINTER(_Grid), vp, vp, ctypes.c_int, d, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_int, PROVIDER, vp, PROVIDER, vp,
                                       ctypes.POINTER(Stats), vp, i32]
        _lib.orc_pcg.argtypes = [ctypes.POINTER(_Grid), vp, vp, ctypes.c_int, d, ctypes.c_int,
                                 ctypes.c_int, ctypes.POINTER(Stats), vp, i32]
        _lib.orc_remove_mean.argtypes = [i64, vp]
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OGrid:
    """Keeps the FP64 coordinate arrays (and the mask) alive for the C
    structure. solid = True takes the grid's mask into the operator (the
    solid-mask mode); by default the mask does not enter it."""

    def __init__(self, g, solid=False):
        self.nx, self.ny = int(g.nx), int(g.ny)
        self.xc, self.yc, self.hx, self.hy = _f64(g.xc), _f64(g.yc), _f64(g.hx), _f64(g.hy)
        self.mask = None
        if solid:
            if getattr(g, "mask", None) is None:
                raise ValueError("the solid-mask mode needs a mask")
            self.mask = np.ascontiguousarray(g.mask, dtype=np.uint8).reshape(self.ny, self.nx)
        self.c = _Grid(self.nx, self.ny, self.xc.ctypes.data, self.yc.ctypes.data,
                       self.hx.ctypes.data, self.hy.ctypes.data,
                       self.mask.ctypes.data if solid else None, 1 if solid else 0)

    @property
    def n(self):
        return self.nx * self.ny


def _og(g):
    return g if isinstance(g, OGrid) else OGrid(g)


def apply(g, x):
    """A x for x of shape [ny, nx] (FP64)."""
    g = _og(g)
    x = _f64(x).reshape(g.ny, g.nx)
    y = np.empty_like(x)
    lib().orc_apply(ctypes.byref(g.c), x.ctypes.data, y.ctypes.data)
    return y


def diag(g):
    g = _og(g)
    d = np.empty((g.ny, g.nx))
    lib().orc_diag(ctypes.byref(g.c), d.ctypes.data)
    return d


def rhs(g, f):
    """b = area * f with the plain mean removed; returns (b, removed_mean).

    f is taken as FP32, the precision the library's boundary accepts."""
    g = _og(g)
    f32 = np.ascontiguousarray(f, dtype=np.float32).reshape(g.ny, g.nx)
    b = np.empty((g.ny, g.nx))
    m = lib().orc_rhs(ctypes.byref(g.c), f32.ctypes.data, b.ctypes.data)
    return b, m


def remove_fluid_mean(g, x):
    """Solid-mask mode's minimum-norm normalisation: subtract the mean over
    the fluid cells from the fluid cells (solid cells unchanged)."""
    x = _f64(x).reshape(int(g.ny), int(g.nx)).copy()
    fl = np.asarray(g.mask).reshape(x.shape) == 0
    x[fl] -= x[fl].mean()
    return x


def remove_mean(x):
    x = _f64(x).copy()
    lib().orc_remove_mean(x.size, x.ctypes.data)
    return x


def _callback(n, fn, err):
    def _cb(ctx, rp, ep):
        try:
            r = np.ctypeslib.as_array(rp, shape=(n.n,)).reshape(n.ny, n.nx).copy()
            e = np.asarray(fn(r), dtype=np.float64).reshape(-1)
            np.ctypeslib.as_array(ep, shape=(n.n,))[:] = e
            return 0
        except Exception as ex:  # reported after the call returns
            err.append(ex)
            return 1
    return _cb


def hybrid(g, b, provider=None, *, x0=None, precond=1, tol=1e-6, tol_kind=0,
           max_iter=10000, num_cg=3, num_dlsm=2, history=False, pc=None):
    """Hybrid solve of Sec. 2.2; ``provider(r) -> e`` maps a residual field
    [ny, nx] to an error direction (None = plain PCG). ``pc(r) -> z`` is a
    preconditioner operator (precond = 2, e.g. ``oracle.mg.Hierarchy.apply``).
    Returns (x, stats, hist)."""
    g = _og(g)
    b = _f64(b).reshape(g.ny, g.nx)
    x = np.zeros_like(b) if x0 is None else _f64(x0).reshape(g.ny, g.nx).copy()
    st = Stats()
    hist = np.full(max_iter + 1, np.nan) if history else None
    hp = hist.ctypes.data if history else None
    cap = max_iter + 1 if history else 0
    err = []
    if precond == 2 and pc is None:
        raise ValueError("precond = 2 needs a preconditioner operator pc")
    cb = PROVIDER(_callback(g, provider, err)) if provider is not None else PROVIDER()
    pcb = PROVIDER(_callback(g, pc, err)) if pc is not None else PROVIDER()
    lib().orc_hybrid_pc(ctypes.byref(g.c), b.ctypes.data, x.ctypes.data, precond, tol, tol_kind,
                        max_iter, num_cg, num_dlsm if provider is not None else 0, cb, None, pcb, None,
                        ctypes.byref(st), hp, cap)
    if err and not isinstance(err[0], FloatingPointError):
        raise err[0]
    if history:
        hist = hist[: st.iters_total + 1]
    return x, st, hist


def pcg(g, b, *, x0=None, precond=1, tol=1e-6, tol_kind=0, max_iter=10000, history=False, pc=None):
    """Textbook PCG (Saad Alg. 9.1) with no, Jacobi or a supplied (pc)
    preconditioner; tol <= 0 runs exactly max_iter iterations."""
    return hybrid(g, b, None, x0=x0, precond=precond, tol=tol, tol_kind=tol_kind,
                  max_iter=max_iter, history=history, pc=pc)
