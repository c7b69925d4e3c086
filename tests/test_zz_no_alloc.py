"""Allocation-free plain solve (ppe_solve_plain_noalloc) through the C-ABI,
against the existing entry point ppe_solve_plain on the same problem: two
calls in a row, the second on a smaller grid, each bit-identical to
ppe_solve_plain (same kernels and order in a fixed device array instead of
the problem's workspace) and at the tolerance on the oracle's FP64 true
residual; the second call changes no device memory use; grids whose state
does not fit the array are rejected before any launch."""
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


def system(nx, ny, seed):
    rng = np.random.default_rng(seed)
    g = inputs.with_ellipse(inputs.random_stretched_grid(nx, ny, rng), rng)
    return g, inputs.grf(g, seed).astype(np.float32)


def true_res(g, f, x):
    b, _ = oracle.rhs(g, f)
    return np.linalg.norm(b - oracle.apply(g, x)) / np.linalg.norm(b)


def test_noalloc_matches_plain_on_consecutive_calls(ppe):
    for k, (nx, ny, tol) in enumerate([(256, 192, 1e-6), (100, 70, 1e-8)]):
        g, f = system(nx, ny, 20 + k)
        prob = ppe.ppe_problem_create(g)
        fd = torch.from_numpy(f).cuda()
        opts = ppe.ppe_solve_opts_default(tol=tol)
        x_ref = torch.zeros((1, ny, nx), dtype=torch.float64, device="cuda")
        st_ref, s_ref = ppe.ppe_solve_plain(prob, fd[None], x_ref, opts)
        x = torch.full((ny, nx), 7.0, dtype=torch.float64, device="cuda")
        opts.zero_x0 = 1
        x_ref0 = torch.zeros_like(x)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        st, s = ppe.ppe_solve_plain_noalloc(prob, fd, x, opts)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        print(f"{nx}x{ny}: iters {s['iters_total']} (plain {s_ref[0]['iters_total']}), "
              f"rel res {s['rel_res_true']:.3e}, scratch {ppe.ppe_noalloc_scratch_bytes(prob)} B")
        assert st == st_ref == ppe.PPE_OK
        for key in ("status", "iters_total", "iters_cg", "reliable_updates", "rel_res_true", "bnorm"):
            assert s[key] == s_ref[0][key], (key, s, s_ref[0])
        xh = x.cpu().numpy()
        np.testing.assert_array_equal(xh, x_ref[0].cpu().numpy())
        assert true_res(g, f, xh) <= tol * 1.001
        if k > 0:
            assert free1 == free0, (free0, free1)
        del x_ref0


def test_noalloc_limits_and_statuses(ppe):
    big = inputs.make_grid(2048, 1024, 1.5)
    pb = ppe.ppe_problem_create(big)
    assert ppe.ppe_noalloc_scratch_bytes(pb) > ppe.PPE_NOALLOC_SCRATCH_BYTES
    fb = torch.zeros((1024, 2048), dtype=torch.float32, device="cuda")
    xb = torch.zeros((1024, 2048), dtype=torch.float64, device="cuda")
    with pytest.raises(ppe.PPEError) as e:
        ppe.ppe_solve_plain_noalloc(pb, fb, xb)
    assert e.value.status == ppe.PPE_ERR_INVALID_ARG
    # the headline size fits
    assert ppe.ppe_noalloc_scratch_bytes(ppe.ppe_problem_create(inputs.make_grid(1024, 1024, 1.75))) \
        <= ppe.PPE_NOALLOC_SCRATCH_BYTES
    g, f = system(64, 48, 5)
    prob = ppe.ppe_problem_create(g)
    f[3, 7] = np.nan
    x = torch.zeros((48, 64), dtype=torch.float64, device="cuda")
    st, s = ppe.ppe_solve_plain_noalloc(prob, torch.from_numpy(f).cuda(), x)
    assert st == ppe.PPE_ERR_NONFINITE and s["status"] == ppe.PPE_ERR_NONFINITE
    # iteration limit, then a clean solve on the same array
    g, f = system(128, 128, 6)
    prob = ppe.ppe_problem_create(g)
    fd = torch.from_numpy(f).cuda()
    x = torch.zeros((128, 128), dtype=torch.float64, device="cuda")
    st, s = ppe.ppe_solve_plain_noalloc(prob, fd, x, ppe.ppe_solve_opts_default(max_iter=40))
    assert st == ppe.PPE_NOT_CONVERGED and s["iters_total"] == 40
    st, s = ppe.ppe_solve_plain_noalloc(prob, fd, x, ppe.ppe_solve_opts_default(zero_x0=1))
    assert st == ppe.PPE_OK and true_res(g, f, x.cpu().numpy()) <= 1e-6 * 1.001
