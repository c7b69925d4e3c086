"""Pins of the oracle's solid-mask mode (CPU only): the masked operator
reduces to the unmasked operator of the fluid sub-grid when the solid region
is a band of whole columns or rows, it is symmetric with the fluid indicator
as its null space and identity rows in solid cells, the right-hand side is
projected over the fluid cells, and PCG on it matches a dense solve."""
import numpy as np
import pytest

from paper_2604_01800_amd import inputs
from oracle import OGrid


def sub_grid(g, i0, i1, j0, j1):
    return inputs.Grid(i1 - i0, j1 - j0, g.xc[i0:i1], g.yc[j0:j1], g.hx[i0:i1], g.hy[j0:j1])


@pytest.mark.parametrize("axis", ["columns", "rows"])
def test_band_mask_reduces_to_sub_grid(orc, axis):
    g = inputs.make_grid(14, 11, 1.6, 0.9)
    mask = np.zeros((11, 14), np.uint8)
    if axis == "columns":
        mask[:, 9:] = 1
        sub = sub_grid(g, 0, 9, 0, 11)
        fl = (slice(None), slice(0, 9))
    else:
        mask[:4, :] = 1
        sub = sub_grid(g, 0, 14, 4, 11)
        fl = (slice(4, None), slice(None))
    g.mask = mask
    og = OGrid(g, solid=True)
    x = np.random.default_rng(1).standard_normal((11, 14))
    y = orc.apply(og, x)
    np.testing.assert_allclose(y[fl], orc.apply(sub, x[fl]), atol=1e-13 * np.abs(y).max())
    np.testing.assert_array_equal(y[mask == 1], x[mask == 1])
    d = orc.diag(og)
    np.testing.assert_allclose(d[fl], orc.diag(sub), rtol=1e-15)
    assert np.all(d[mask == 1] == 1.0)


def ellipse_grid(n, seed):
    g = inputs.make_grid(n, n, 1.5)
    g.mask = inputs.ellipse_mask(g.xc, g.yc, (0.5, 0.45, 0.2, 0.12, 0.6)).astype(np.uint8)
    assert g.mask.any()
    return g


def test_symmetry_null_space_and_rhs(orc):
    g = ellipse_grid(24, 0)
    og = OGrid(g, solid=True)
    rng = np.random.default_rng(2)
    u, v = rng.standard_normal((2, 24, 24))
    Au, Av = orc.apply(og, u), orc.apply(og, v)
    assert abs(np.sum(u * Av) - np.sum(v * Au)) <= 1e-13 * np.abs(Au).max() * u.size
    ind = (g.mask == 0).astype(np.float64)
    assert np.abs(orc.apply(og, ind)).max() <= 1e-13 * np.abs(orc.diag(og)).max()
    b, m = orc.rhs(og, inputs.gaussian_bumps(g, 3).astype(np.float32))
    assert np.all(b[g.mask == 1] == 0.0)
    assert abs(b[g.mask == 0].sum()) <= 1e-14 * np.abs(b).sum()


def test_pcg_matches_dense_solve(orc):
    g = ellipse_grid(18, 1)
    og = OGrid(g, solid=True)
    b, _ = orc.rhs(og, inputs.gaussian_bumps(g, 4).astype(np.float32))
    N = g.nx * g.ny
    A = np.stack([orc.apply(og, e.reshape(g.ny, g.nx)).reshape(-1) for e in np.eye(N)], axis=1)
    xd = (np.linalg.pinv(A) @ b.reshape(-1)).reshape(g.ny, g.nx)
    x, st, _ = orc.pcg(og, b, tol=1e-13, max_iter=5000)
    assert st.converged
    x = orc.remove_fluid_mean(g, x)
    assert np.abs(x[g.mask == 1]).max() == 0.0
    np.testing.assert_allclose(x, xd, atol=1e-10 * np.abs(xd).max())
