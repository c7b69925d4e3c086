"""Seeded synthetic inputs: stretched grids, obstacle masks, right-hand-side
fields and network parameter draws.

This module is shared by the tests, the benchmark and the oracle checks. It
draws random numbers and lays out coordinates; it holds none of the solver's
arithmetic (no operator, no projection, no iteration, no network layer).

Recipes (all on the unit square, cell-centred):

* tanh stretching: faces x(xi) = 1/2 [1 + tanh(beta (2 xi - 1)) / tanh(beta)],
  xi = i/n, clustered at both walls; centres are face midpoints, widths are
  face differences. beta = 0 is the uniform grid. The max/min width ratio is
  close to cosh(beta)^2, so beta = 1.0, 2.35 and 2.5 stand in for the paper's
  spacing ratios 2.3, 28 and 41 (Table 1).
* Gaussian bumps: f = sum_k A_k exp(-|x - c_k|^2 / (2 w_k^2)), c ~ U[0,1]^2,
  w ~ U[0.02, 0.1], A ~ N(0, 1).
* Gaussian random field with squared-exponential covariance
  exp(-r^2 / (2 l^2)) through J random Fourier features (Rahimi & Recht 2007):
  g(x) = sqrt(2/J) sum_j a_j cos(w_j . x + phi_j), w_j ~ N(0, I / l^2),
  phi_j ~ U[0, 2 pi), a_j ~ N(0, 1).
* Ellipse obstacle: centre ~ U[0.2, 0.8]^2, semi-axes ~ U[0.05, 0.15],
  angle ~ U[0, pi); a cell is solid when its centre lies inside.
"""
from __future__ import annotations

import dataclasses

import numpy as np


def tanh_faces(n: int, beta: float) -> np.ndarray:
    """Face coordinates of an n-cell tanh-stretched 1D grid on [0, 1]."""
    xi = np.arange(n + 1, dtype=np.float64) / n
    if beta == 0.0:
        return xi
    f = 0.5 * (1.0 + np.tanh(beta * (2.0 * xi - 1.0)) / np.tanh(beta))
    f[0], f[-1] = 0.0, 1.0
    return f


@dataclasses.dataclass
class Grid:
    """A tensor-product cell-centred grid with an optional solid mask."""

    nx: int
    ny: int
    xc: np.ndarray  # [nx] cell centres, strictly increasing
    yc: np.ndarray  # [ny]
    hx: np.ndarray  # [nx] cell widths
    hy: np.ndarray  # [ny]
    mask: np.ndarray | None = None  # [ny, nx] uint8, 1 = solid
    beta_x: float = 0.0
    beta_y: float = 0.0
    ellipse: tuple | None = None  # (cx, cy, a, b, theta) when the mask is an ellipse

    @property
    def n(self) -> int:
        return self.nx * self.ny


def make_grid(nx: int, ny: int, beta_x: float, beta_y: float | None = None) -> Grid:
    if beta_y is None:
        beta_y = beta_x
    fx = tanh_faces(nx, beta_x)
    fy = tanh_faces(ny, beta_y)
    return Grid(nx, ny, 0.5 * (fx[1:] + fx[:-1]), 0.5 * (fy[1:] + fy[:-1]),
                np.diff(fx), np.diff(fy), None, float(beta_x), float(beta_y))


def ellipse_params(rng: np.random.Generator, semi_lo=0.05, semi_hi=0.15):
    cx, cy = rng.uniform(0.2, 0.8, size=2)
    a, b = rng.uniform(semi_lo, semi_hi, size=2)
    theta = rng.uniform(0.0, np.pi)
    return float(cx), float(cy), float(a), float(b), float(theta)


def ellipse_mask(xc: np.ndarray, yc: np.ndarray, params) -> np.ndarray:
    cx, cy, a, b, theta = params
    X = xc[None, :] - cx
    Y = yc[:, None] - cy
    c, s = np.cos(theta), np.sin(theta)
    u = c * X + s * Y
    v = -s * X + c * Y
    return ((u / a) ** 2 + (v / b) ** 2 <= 1.0).astype(np.uint8)


def with_ellipse(g: Grid, rng: np.random.Generator) -> Grid:
    p = ellipse_params(rng)
    return dataclasses.replace(g, mask=ellipse_mask(g.xc, g.yc, p), ellipse=p)


def random_stretched_grid(nx: int, ny: int, rng: np.random.Generator,
                          beta_lo=1.0, beta_hi=2.5, mask=True) -> Grid:
    bx, by = rng.uniform(beta_lo, beta_hi, size=2)
    g = make_grid(nx, ny, float(bx), float(by))
    return with_ellipse(g, rng) if mask else g


def gaussian_bumps(g: Grid, seed: int, k: int = 8) -> np.ndarray:
    """Sum of k Gaussian bumps at the cell centres, [ny, nx] float64."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, 1.0, size=(k, 2))
    w = rng.uniform(0.02, 0.1, size=k)
    A = rng.standard_normal(k)
    f = np.zeros((g.ny, g.nx))
    for m in range(k):
        ex = np.exp(-((g.xc - c[m, 0]) ** 2) / (2 * w[m] ** 2))
        ey = np.exp(-((g.yc - c[m, 1]) ** 2) / (2 * w[m] ** 2))
        f += A[m] * np.outer(ey, ex)
    return f


def grf_features(rng: np.random.Generator, ell: float = 0.05, J: int = 512):
    """Random Fourier feature draws (w [J,2], phi [J], a [J])."""
    w = rng.standard_normal((J, 2)) / ell
    phi = rng.uniform(0.0, 2.0 * np.pi, size=J)
    a = rng.standard_normal(J)
    return w, phi, a


def grf_eval(xc: np.ndarray, yc: np.ndarray, feats) -> np.ndarray:
    """Evaluate the feature sum at the tensor grid, [ny, nx] float64.

    cos(wx x + wy y + phi) is split as cos(wx x + phi) cos(wy y) -
    sin(wx x + phi) sin(wy y), so the sum is two [ny, J] x [J, nx] products.
    """
    w, phi, a = feats
    J = w.shape[0]
    ax = np.outer(xc, w[:, 0]) + phi[None, :]  # [nx, J]
    ay = np.outer(yc, w[:, 1])  # [ny, J]
    s = np.sqrt(2.0 / J)
    return s * ((np.cos(ay) * a) @ np.cos(ax).T - (np.sin(ay) * a) @ np.sin(ax).T)


def grf(g: Grid, seed: int, ell: float = 0.05, J: int = 512) -> np.ndarray:
    return grf_eval(g.xc, g.yc, grf_features(np.random.default_rng(seed), ell, J))


def travelling_grf(g: Grid, seed: int, steps: int, shift: float = 0.001,
                   direction=(0.95, 0.31), ell: float = 0.05, J: int = 512) -> np.ndarray:
    """Source sequence for consecutive solves on one grid, [steps, ny, nx] float32.

    The grf(g, seed) pattern carried along a unit `direction` by `shift` domain
    lengths per step, as a pressure source does in a flow that advects it
    between time steps: step t is the same feature sum with every phase phi
    moved to phi - t * shift * (w . direction), i.e. the step-0 field read at
    (x, y) - t * shift * direction. Step 0 equals grf(g, seed)."""
    w, phi, a = grf_features(np.random.default_rng(seed), ell, J)
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    k = w @ d
    out = np.empty((steps, g.ny, g.nx), dtype=np.float32)
    for t in range(steps):
        out[t] = grf_eval(g.xc, g.yc, (w, phi - t * shift * k, a))
    return out
