"""Python binding of the C-ABI in include/ppe.h (argument marshalling only).

Every function has the name of the C entry point it calls. Device arrays are
torch tensors on the current HIP device (torch supplies memory and streams
only; all arithmetic runs in the library's HIP kernels). The library must be
built (``python -m paper_2604_01800_amd.build``); loading fails loudly if it
is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libppe_hip.so")

PPE_OK, PPE_NOT_CONVERGED = 0, 1
PPE_ERR_INVALID_ARG, PPE_ERR_SHAPE, PPE_ERR_UNSUPPORTED, PPE_ERR_HIP, PPE_ERR_NONFINITE = -1, -2, -3, -4, -5
PPE_PC_NONE, PPE_PC_JACOBI, PPE_PC_MG, PPE_PC_IC = 0, 1, 2, 3
PPE_MASK_DIBPM, PPE_MASK_SOLID = 0, 1
PPE_LOSS_RESIDUAL, PPE_LOSS_SUPERVISED, PPE_LOSS_ANORM = 0, 1, 2
PPE_TOL_RELATIVE, PPE_TOL_ABSOLUTE = 0, 1
PPE_PCG_AUTO, PPE_PCG_SINGLE_REDUCTION, PPE_PCG_TWO_PHASE, PPE_PCG_TWO_STEP = 0, 1, 2, 3
PPE_DIR_NET, PPE_DIR_ZERO, PPE_DIR_JACOBI, PPE_DIR_NAN, PPE_DIR_ONES = 0, 1, 2, 3, 4


class PPEError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ppe status {status}: {msg}")
        self.status = status


class ppe_grid_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("xc", ctypes.c_void_p), ("yc", ctypes.c_void_p),
                ("hx", ctypes.c_void_p), ("hy", ctypes.c_void_p),
                ("mask", ctypes.c_void_p), ("mask_mode", ctypes.c_int32)]


class ppe_solve_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("tol_kind", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("num_cg", ctypes.c_int32), ("num_dlsm", ctypes.c_int32),
                ("direction", ctypes.c_int32), ("reliable_delta", ctypes.c_double),
                ("rows_per_wave", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("zero_x0", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("mg_levels", ctypes.c_int32), ("record_history", ctypes.c_int32)]


class ppe_tune_result(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("rows_per_wave", ctypes.c_int32),
                ("us_per_iter", (ctypes.c_double * 6) * 3)]


PPE_NET_MAX_LAUNCHES = 64


class ppe_net_tune_result(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("tile", ctypes.c_int32 * PPE_NET_MAX_LAUNCHES),
                ("us32", ctypes.c_float * PPE_NET_MAX_LAUNCHES), ("us64", ctypes.c_float * PPE_NET_MAX_LAUNCHES)]


class ppe_solve_stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters_total", ctypes.c_int32), ("iters_cg", ctypes.c_int32),
                ("iters_dlsm", ctypes.c_int32), ("dlsm_rejected", ctypes.c_int32),
                ("reliable_updates", ctypes.c_int32), ("rel_res_true", ctypes.c_double),
                ("abs_res_true", ctypes.c_double), ("bnorm", ctypes.c_double),
                ("rhs_mean_removed", ctypes.c_double), ("ms_total", ctypes.c_double), ("ms_device", ctypes.c_double),
                ("ms_pcg", ctypes.c_double), ("ms_net", ctypes.c_double), ("ms_dlsm", ctypes.c_double),
                ("history", ctypes.c_void_p), ("history_cap", ctypes.c_int32), ("history_len", ctypes.c_int32)]

    def as_dict(self, hist=None):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("history", "history_cap")}
        d["history"] = None if hist is None else hist[: self.history_len].copy()
        return d


HISTORY_CAP_MAX = 1 << 22


def _stats_array(nb, opts):
    """Stats structs for nb solves, with a history buffer per solve when the
    options ask for the residual history. Returns (array, buffers)."""
    stats = (ppe_solve_stats * max(nb, 1))()
    bufs = [None] * max(nb, 1)
    if opts is not None and opts.record_history:
        cap = int(min(max(opts.max_iter, 0) + 1, HISTORY_CAP_MAX))
        for i in range(nb):
            bufs[i] = np.zeros(cap, dtype=np.float64)
            stats[i].history = bufs[i].ctypes.data
            stats[i].history_cap = cap
    return stats, bufs


class ppe_net_config(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("base_channels", ctypes.c_int32), ("basis", ctypes.c_int32),
                ("trunk_width", ctypes.c_int32), ("trunk_hidden", ctypes.c_int32),
                ("phi_hidden", ctypes.c_int32), ("use_eta", ctypes.c_int32), ("use_spacing", ctypes.c_int32)]


class ppe_train_opts(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("seed", ctypes.c_uint64), ("step", ctypes.c_int64),
                ("grf_len_lo", ctypes.c_float), ("grf_len_hi", ctypes.c_float), ("grf_features", ctypes.c_int32),
                ("clip_norm", ctypes.c_float), ("sam_rho", ctypes.c_float), ("loss_kind", ctypes.c_int32)]


# name -> (restype, argtypes); every symbol declared in include/ppe.h
_vp, _i32, _i64, _u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
_P = ctypes.POINTER
SIGNATURES = {
    "ppe_problem_create": (_i32, [_P(ppe_grid_desc), _vp, _P(_vp)]),
    "ppe_problem_destroy": (None, [_vp]),
    "ppe_solve_opts_default": (None, [_P(ppe_solve_opts)]),
    "ppe_apply_f32": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "ppe_apply_f64": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "ppe_rhs_to_source": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "ppe_solve_plain": (_i32, [_vp, _i32, _vp, _vp, _P(ppe_solve_opts), _vp, _vp]),
    "ppe_apply_precond": (_i32, [_vp, _i32, _vp, _vp, _P(ppe_solve_opts), _vp]),
    "ppe_solve_hybrid": (_i32, [_vp, _vp, _i32, _vp, _vp, _P(ppe_solve_opts), _vp, _vp]),
    "ppe_net_config_default": (None, [_P(ppe_net_config)]),
    "ppe_net_create": (_i32, [_P(ppe_net_config), _u64, _P(_vp)]),
    "ppe_net_destroy": (None, [_vp]),
    "ppe_net_num_params": (_i64, [_vp]),
    "ppe_net_set_params": (_i32, [_vp, _vp, _i64]),
    "ppe_net_get_params": (_i32, [_vp, _vp, _i64]),
    "ppe_net_save": (_i32, [_vp, ctypes.c_char_p]),
    "ppe_net_load": (_i32, [_vp, ctypes.c_char_p]),
    "ppe_net_forward": (_i32, [_vp, _vp, _i32, _vp, _vp, _vp]),
    "ppe_net_forward_batch": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp]),
    "ppe_tune_net": (_i32, [_vp, _vp, _i32, _i32, _P(ppe_net_tune_result), _vp]),
    "ppe_net_train_step": (_i32, [_vp, _i32, _vp, _vp, _vp, _P(ppe_train_opts), _vp, _vp, _vp]),
    "ppe_profile_pcg": (_i32, [_vp, _i32, _vp, _vp, _P(ppe_solve_opts), _i32, _vp, _vp]),
    "ppe_profile_copy": (_i32, [_vp, _vp, _i64, _i32, _vp, _vp]),
    "ppe_solve_batch": (_i32, [_i32, _vp, _vp, _vp, _vp, _P(ppe_solve_opts), _vp, _vp]),
    "ppe_generate_rhs": (_i32, [_i32, _vp, _P(ppe_train_opts), _vp, _vp]),
    "ppe_generate_grid": (_i32, [_i32, _i32, _u64, _u64, _i32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "ppe_ritz_create": (_i32, [_vp, _i32, _vp, _P(_vp), _vp]),
    "ppe_ritz_info": (_i32, [_vp, _P(_i32), _vp, _vp, _vp]),
    "ppe_ritz_rhs": (_i32, [_vp, _i32, _u64, _i64, ctypes.c_double, ctypes.c_double, _vp, _vp]),
    "ppe_ritz_destroy": (None, [_vp]),
    "ppe_tridiag_eigh": (_i32, [_i32, _vp, _vp, _vp, _vp]),
    "ppe_tune_pcg": (_i32, [_vp, _i32, _vp, _vp, _i32, _P(ppe_tune_result), _vp]),
    "ppe_set_tuning": (_i32, [_vp, _i32, _i32, _i32]),
    "ppe_get_tuning": (_i32, [_vp, _i32, _P(ctypes.c_int32), _P(ctypes.c_int32)]),
    "ppe_noalloc_scratch_bytes": (_i64, [_vp]),
    "ppe_solve_plain_noalloc": (_i32, [_vp, _vp, _vp, _P(ppe_solve_opts), _vp, _vp]),
    "ppe_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load the built HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2604_01800_amd.build`")
        # torch first: it brings its own HIP runtime (soname libamdhip64.so.7),
        # and the library must bind to that one, the runtime of the device
        # memory and streams it is handed. Loaded the other way round, the
        # process would run torch on the system runtime, and the library's
        # allocations fail after torch initialises the device.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name, None)
            if fn is None:
                raise ImportError(f"{LIB_PATH} does not export {name}: rebuild the library")
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    L = lib()
    return {n for n in SIGNATURES if hasattr(L, n)}


def _check(st, allow=(PPE_OK,)):
    if st not in allow:
        raise PPEError(st, lib().ppe_last_error().decode())
    return st


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Problem:
    """Owns a ppe_problem handle (one grid)."""

    def __init__(self, grid, mask_mode=PPE_MASK_DIBPM, stream=None):
        self.nx, self.ny = int(grid.nx), int(grid.ny)
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (grid.xc, grid.yc, grid.hx, grid.hy)]
        mask = None if getattr(grid, "mask", None) is None else np.ascontiguousarray(grid.mask, dtype=np.uint8)
        d = ppe_grid_desc(self.nx, self.ny, *[a.ctypes.data for a in arrs],
                          mask.ctypes.data if mask is not None else None, mask_mode)
        h = ctypes.c_void_p()
        s = None
        if stream is not None:
            s = ctypes.c_void_p(stream.cuda_stream)
        _check(lib().ppe_problem_create(ctypes.byref(d), s, ctypes.byref(h)))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.ppe_problem_destroy(h)
            self.handle = None


def ppe_problem_create(grid, mask_mode=PPE_MASK_DIBPM, stream=None) -> Problem:
    return Problem(grid, mask_mode, stream)


def ppe_solve_opts_default(**kw) -> ppe_solve_opts:
    o = ppe_solve_opts()
    lib().ppe_solve_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _nb(t, prob):
    if t.dim() == 2:
        nb = 1
        shape = tuple(t.shape)
    else:
        nb = t.shape[0]
        shape = tuple(t.shape[1:])
    if shape != (prob.ny, prob.nx):
        raise ValueError(f"field shape {shape} != ({prob.ny}, {prob.nx})")
    return nb


def ppe_apply_f32(prob: Problem, x, y, stream=None):
    import torch
    nb = _nb(x, prob)
    _check(lib().ppe_apply_f32(prob.handle, nb, _dev(x, torch.float32, "x"), _dev(y, torch.float32, "y"),
                               _stream(stream)))


def ppe_apply_f64(prob: Problem, x, y, stream=None):
    import torch
    nb = _nb(x, prob)
    _check(lib().ppe_apply_f64(prob.handle, nb, _dev(x, torch.float64, "x"), _dev(y, torch.float64, "y"),
                               _stream(stream)))


def ppe_rhs_to_source(prob: Problem, b, f, stream=None):
    """f = b / (cell area) (float32 device arrays [nb, ny, nx] or [ny, nx]):
    the source whose right-hand side is b. Enqueued, not synchronised."""
    import torch
    nb = _nb(b, prob)
    _nb(f, prob)
    _check(lib().ppe_rhs_to_source(prob.handle, nb, _dev(b, torch.float32, "b"), _dev(f, torch.float32, "f"),
                                   _stream(stream)))


def ppe_apply_precond(prob: Problem, r, z, opts=None, stream=None):
    """z = M^-1 r (float32 device arrays [nb, ny, nx] or [ny, nx]) for the
    preconditioner opts.precond selects."""
    import torch
    nb = _nb(r, prob)
    if _nb(z, prob) != nb:
        raise ValueError("r and z batch sizes differ")
    opts = opts or ppe_solve_opts_default()
    _check(lib().ppe_apply_precond(prob.handle, nb, _dev(r, torch.float32, "r"), _dev(z, torch.float32, "z"),
                                   ctypes.byref(opts), _stream(stream)))


def ppe_solve_plain(prob: Problem, f, x, opts=None, stream=None):
    """Returns (status, [stats dict per solve])."""
    import torch
    nb = _nb(f, prob)
    if _nb(x, prob) != nb:
        raise ValueError("f and x batch sizes differ")
    opts = opts or ppe_solve_opts_default()
    stats, bufs = _stats_array(nb, opts)
    st = lib().ppe_solve_plain(prob.handle, nb, _dev(f, torch.float32, "f"), _dev(x, torch.float64, "x"),
                               ctypes.byref(opts), ctypes.cast(stats, ctypes.c_void_p), _stream(stream))
    _check(st, (PPE_OK, PPE_NOT_CONVERGED, PPE_ERR_NONFINITE))
    return st, [stats[i].as_dict(bufs[i]) for i in range(nb)]


def ppe_solve_plain_noalloc(prob: Problem, f, x, opts=None, stream=None):
    """Allocation-free plain solve of one right-hand side (f: device float32
    [ny, nx] or [1, ny, nx]; x: device float64 of the same shape). Returns
    (status, stats dict)."""
    import torch
    if _nb(f, prob) != 1 or _nb(x, prob) != 1:
        raise ValueError("the allocation-free solve takes one right-hand side")
    opts = opts or ppe_solve_opts_default()
    stats, bufs = _stats_array(1, opts)
    st = lib().ppe_solve_plain_noalloc(prob.handle, _dev(f, torch.float32, "f"), _dev(x, torch.float64, "x"),
                                       ctypes.byref(opts), ctypes.cast(stats, ctypes.c_void_p), _stream(stream))
    _check(st, (PPE_OK, PPE_NOT_CONVERGED, PPE_ERR_NONFINITE))
    return st, stats[0].as_dict(bufs[0])


def ppe_noalloc_scratch_bytes(prob: Problem) -> int:
    return int(lib().ppe_noalloc_scratch_bytes(prob.handle))


PPE_NOALLOC_SCRATCH_BYTES = 32 * 1024 * 1024


def ppe_profile_pcg(prob: Problem, f, x, opts=None, reps=50, stream=None):
    """Average ms of one phase-A and one phase-B launch (HIP events)."""
    import torch
    nb = _nb(f, prob)
    opts = opts or ppe_solve_opts_default()
    out = (ctypes.c_double * 2)()
    _check(lib().ppe_profile_pcg(prob.handle, nb, _dev(f, torch.float32, "f"), _dev(x, torch.float64, "x"),
                                 ctypes.byref(opts), reps, ctypes.cast(out, ctypes.c_void_p), _stream(stream)))
    return out[0], out[1]


def ppe_tune_pcg(prob: Problem, f, x, reps=20, stream=None):
    """Times every iteration form x tile height on (f, x) (x is overwritten),
    stores the fastest in the problem for this batch size and returns
    {"variant", "rows_per_wave", "us_per_iter": {(form, rows): us}}."""
    import torch
    nb = _nb(f, prob)
    res = ppe_tune_result()
    _check(lib().ppe_tune_pcg(prob.handle, nb, _dev(f, torch.float32, "f"), _dev(x, torch.float64, "x"), reps,
                              ctypes.byref(res), _stream(stream)))
    forms = ("single", "two_phase", "two_step")
    table = {(forms[v], r): res.us_per_iter[v][k] for v in range(3) for k, r in enumerate((2, 4, 8, 16, 20, 24))
             if res.us_per_iter[v][k] > 0}
    return {"variant": res.variant, "rows_per_wave": res.rows_per_wave, "us_per_iter": table}


def ppe_set_tuning(prob: Problem, nb: int, variant: int, rows_per_wave: int):
    _check(lib().ppe_set_tuning(prob.handle, nb, variant, rows_per_wave))


def ppe_get_tuning(prob: Problem, nb: int):
    v, r = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().ppe_get_tuning(prob.handle, nb, ctypes.byref(v), ctypes.byref(r)))
    return v.value, r.value


def ppe_profile_copy(src, dst, reps=20, stream=None):
    """Average ms of a device copy of src.nbytes bytes into dst."""
    if src.nbytes != dst.nbytes:
        raise ValueError("src and dst sizes differ")
    out = (ctypes.c_double * 1)()
    _check(lib().ppe_profile_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                  src.nbytes, reps, ctypes.cast(out, ctypes.c_void_p), _stream(stream)))
    return out[0]


def ppe_net_config_default(**kw) -> ppe_net_config:
    c = ppe_net_config()
    lib().ppe_net_config_default(ctypes.byref(c))
    for k, v in kw.items():
        if not hasattr(c, k):
            raise KeyError(k)
        setattr(c, k, v)
    return c


class Net:
    """Owns a ppe_net handle (DeepONet weights and optimiser state)."""

    def __init__(self, cfg=None, seed=0):
        cfg = cfg or ppe_net_config_default()
        h = ctypes.c_void_p()
        _check(lib().ppe_net_create(ctypes.byref(cfg), seed, ctypes.byref(h)))
        self.handle = h
        self.cfg = cfg

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.ppe_net_destroy(h)
            self.handle = None


def ppe_net_create(cfg=None, seed=0) -> Net:
    return Net(cfg, seed)


def ppe_net_num_params(net: Net) -> int:
    return int(lib().ppe_net_num_params(net.handle))


def ppe_net_set_params(net: Net, flat):
    a = np.ascontiguousarray(flat, dtype=np.float32)
    _check(lib().ppe_net_set_params(net.handle, a.ctypes.data, a.size))


def ppe_net_get_params(net: Net) -> np.ndarray:
    n = ppe_net_num_params(net)
    a = np.empty(n, dtype=np.float32)
    _check(lib().ppe_net_get_params(net.handle, a.ctypes.data, n))
    return a


def ppe_net_save(net: Net, path: str):
    _check(lib().ppe_net_save(net.handle, path.encode()))


def ppe_net_load(net: Net, path: str):
    _check(lib().ppe_net_load(net.handle, path.encode()))


def ppe_net_forward(net: Net, prob: Problem, r, y, stream=None):
    import torch
    nb = _nb(r, prob)
    _check(lib().ppe_net_forward(net.handle, prob.handle, nb, _dev(r, torch.float32, "r"),
                                 _dev(y, torch.float32, "y"), _stream(stream)))


def ppe_tune_net(net: Net, prob: Problem, nb: int = 1, reps: int = 20, stream=None):
    """Tile-width tuning of the network forward on prob's grid for batch
    size nb (stored in the problem); returns the per-launch choices
    {k: (tile, us32, us64)} for the launches that have a choice."""
    res = ppe_net_tune_result()
    _check(lib().ppe_tune_net(net.handle, prob.handle, nb, reps, ctypes.byref(res), _stream(stream)))
    return {k: (res.tile[k], res.us32[k], res.us64[k]) for k in range(res.n) if res.tile[k]}


def ppe_net_forward_batch(net: Net, probs, rs, ys, stream=None):
    """The forward on one field of each of len(probs) grids of any sizes, one
    grouped launch per layer. rs[i], ys[i]: device float32 [ny_i, nx_i]
    (or [1, ny_i, nx_i])."""
    import torch
    n = len(probs)
    if len(rs) != n or len(ys) != n:
        raise ValueError("one input and one output per problem")
    for p, r, y in zip(probs, rs, ys):
        for t in (r, y):
            if t.numel() != p.nx * p.ny:
                raise ValueError("array size does not match its grid")
    parr = (ctypes.c_void_p * n)(*[p.handle.value for p in probs])
    rarr = (ctypes.c_void_p * n)(*[_dev(r, torch.float32, "r") for r in rs])
    yarr = (ctypes.c_void_p * n)(*[_dev(y, torch.float32, "y") for y in ys])
    _check(lib().ppe_net_forward_batch(net.handle, n, ctypes.cast(parr, ctypes.c_void_p),
                                       ctypes.cast(rarr, ctypes.c_void_p), ctypes.cast(yarr, ctypes.c_void_p),
                                       _stream(stream)))


def ppe_solve_hybrid(prob: Problem, net, f, x, opts=None, stream=None):
    """Hybrid CG / line-search solve; net may be None for a test direction.
    Returns (status, [stats dict per solve])."""
    import torch
    nb = _nb(f, prob)
    if _nb(x, prob) != nb:
        raise ValueError("f and x batch sizes differ")
    opts = opts or ppe_solve_opts_default()
    stats, bufs = _stats_array(nb, opts)
    st = lib().ppe_solve_hybrid(prob.handle, net.handle if net is not None else None, nb,
                                _dev(f, torch.float32, "f"), _dev(x, torch.float64, "x"), ctypes.byref(opts),
                                ctypes.cast(stats, ctypes.c_void_p), _stream(stream))
    _check(st, (PPE_OK, PPE_NOT_CONVERGED, PPE_ERR_NONFINITE))
    return st, [stats[i].as_dict(bufs[i]) for i in range(nb)]


def ppe_train_opts_default(**kw) -> ppe_train_opts:
    o = ppe_train_opts(1e-3, 0.9, 0.999, 1e-8, 0, 0, 0.05, 0.5, 512, 0.0, 0.0, PPE_LOSS_RESIDUAL)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def ppe_solve_batch(probs, fs, xs, opts=None, stream=None, net=None):
    """Solves of one right-hand side on each of len(probs) grids of any sizes:
    plain PCG batched per iteration, or with a network the hybrid solve, its
    rounds advanced in lock step. fs[i]: device float32 [ny_i, nx_i] (or
    [1, ny_i, nx_i]); xs[i]: device float64 of the same shape. Returns
    (status, list of stats dicts)."""
    import torch
    n = len(probs)
    if len(fs) != n or len(xs) != n:
        raise ValueError("one source and one solution per problem")
    for p, f, x in zip(probs, fs, xs):
        for t in (f, x):
            if t.numel() != p.nx * p.ny:
                raise ValueError("array size does not match its grid")
    parr = (ctypes.c_void_p * n)(*[p.handle.value for p in probs])
    farr = (ctypes.c_void_p * n)(*[_dev(f, torch.float32, "f") for f in fs])
    xarr = (ctypes.c_void_p * n)(*[_dev(x, torch.float64, "x") for x in xs])
    opts = opts or ppe_solve_opts_default()
    stats, bufs = _stats_array(n, opts)
    st = lib().ppe_solve_batch(n, ctypes.cast(parr, ctypes.c_void_p), net.handle if net is not None else None,
                               ctypes.cast(farr, ctypes.c_void_p),
                               ctypes.cast(xarr, ctypes.c_void_p), ctypes.byref(opts),
                               ctypes.cast(stats, ctypes.c_void_p), _stream(stream))
    _check(st, allow=(PPE_OK, PPE_NOT_CONVERGED, PPE_ERR_NONFINITE))
    return st, [stats[i].as_dict(bufs[i]) for i in range(n)]


def ppe_generate_grid(nx, ny, seed, step, sample, mask=True):
    """Grid of fabricated training system `sample` at step `step` (drawn by the
    library on the host); returns an inputs.Grid with its draws recorded."""
    import numpy as np
    from . import inputs
    xc, yc, hx, hy = np.empty(nx), np.empty(ny), np.empty(nx), np.empty(ny)
    m = np.empty((ny, nx), dtype=np.uint8) if mask else None
    par = np.empty(7)
    _check(lib().ppe_generate_grid(nx, ny, seed, step, sample, xc.ctypes.data, yc.ctypes.data, hx.ctypes.data,
                                   hy.ctypes.data, m.ctypes.data if mask else None, par.ctypes.data))
    return inputs.Grid(nx, ny, xc, yc, hx, hy, m, float(par[0]), float(par[1]),
                       tuple(float(v) for v in par[2:]) if mask else None)


def ppe_generate_rhs(probs, opts, R, stream=None):
    """Fabricated right-hand sides on the device into R (float32 [nb, ny, nx])."""
    import torch
    nb = len(probs)
    if R.dim() != 3 or R.shape[0] != nb:
        raise ValueError("R must be [nb, ny, nx] with one sample per problem")
    for p in probs:
        _nb(R[0], p)
    arr = (ctypes.c_void_p * nb)(*[p.handle.value for p in probs])
    _check(lib().ppe_generate_rhs(nb, ctypes.cast(arr, ctypes.c_void_p), ctypes.byref(opts),
                                  _dev(R, torch.float32, "R"), _stream(stream)))


def ppe_net_train_step(net: Net, probs, R, opts=None, want_grad=False, stream=None, target=None):
    """One Adam step (lr = 0: gradient only). probs: list of Problem (one grid per sample),
    R: device float32 [nb, ny, nx], or None to generate the batch on the device from
    opts (seed, step, length scales, features); target: device float64 [nb, ny, nx]
    for the supervised loss. Returns (loss, grad ndarray or None)."""
    import torch
    nb = len(probs)
    if R is not None:
        if R.dim() != 3 or R.shape[0] != nb:
            raise ValueError("R must be [nb, ny, nx] with one sample per problem")
        for p in probs:
            _nb(R[0], p)
    arr = (ctypes.c_void_p * nb)(*[p.handle.value for p in probs])
    opts = opts or ppe_train_opts_default()
    loss = ctypes.c_float()
    grad = np.empty(ppe_net_num_params(net), dtype=np.float32) if want_grad else None
    Rp = None if R is None else _dev(R, torch.float32, "R")
    Tp = None
    if target is not None:
        if target.dim() != 3 or target.shape[0] != nb:
            raise ValueError("target must be [nb, ny, nx]")
        for p in probs:
            _nb(target[0], p)
        Tp = _dev(target, torch.float64, "target")
    _check(lib().ppe_net_train_step(net.handle, nb, ctypes.cast(arr, ctypes.c_void_p), Rp, Tp,
                                    ctypes.byref(opts), ctypes.byref(loss),
                                    grad.ctypes.data if want_grad else None, _stream(stream)))
    return float(loss.value), grad


class Ritz:
    """Owns a ppe_ritz handle: m Lanczos steps on a problem's operator from the
    device FP64 start vector v0 [ny, nx] (Sec. 2.3, Eq. 14)."""

    def __init__(self, prob: Problem, m: int, v0, stream=None):
        import torch
        if v0.numel() != prob.nx * prob.ny:
            raise ValueError("v0 must hold one value per cell")
        h = ctypes.c_void_p()
        _check(lib().ppe_ritz_create(prob.handle, m, _dev(v0, torch.float64, "v0"), ctypes.byref(h),
                                     _stream(stream)))
        self.handle = h
        self.nx, self.ny = prob.nx, prob.ny

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.ppe_ritz_destroy(h)
            self.handle = None


def ppe_ritz_info(r: Ritz):
    """(alpha [m], beta [m - 1], theta [m] ascending) as numpy arrays."""
    m = ctypes.c_int32()
    _check(lib().ppe_ritz_info(r.handle, ctypes.byref(m), None, None, None))
    a, b, t = np.empty(m.value), np.empty(max(m.value - 1, 0)), np.empty(m.value)
    _check(lib().ppe_ritz_info(r.handle, None, a.ctypes.data, b.ctypes.data if b.size else None, t.ctypes.data))
    return a, b, t


def ppe_ritz_rhs(r: Ritz, R, seed=0, step=0, b=0.6, scale=1.0, stream=None):
    """Fills the device FP32 tensor R [nb, ny, nx] with training vectors
    (Eqs. 15-16) of L2 norm `scale`."""
    import torch
    if R.dim() != 3 or tuple(R.shape[1:]) != (r.ny, r.nx):
        raise ValueError("R must be [nb, ny, nx] on the Ritz basis's grid")
    _check(lib().ppe_ritz_rhs(r.handle, R.shape[0], seed, step, b, scale, _dev(R, torch.float32, "R"),
                              _stream(stream)))


def ppe_tridiag_eigh(alpha, beta):
    """Host eigen-decomposition of a symmetric tridiagonal matrix: (theta, U)."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    n = a.size
    t, U = np.empty(n), np.empty((n, n))
    _check(lib().ppe_tridiag_eigh(n, a.ctypes.data, b.ctypes.data if b.size else None, t.ctypes.data, U.ctypes.data))
    return t, U
