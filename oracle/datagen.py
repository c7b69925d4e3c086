"""TEST INFRASTRUCTURE — reference of the on-device training-data generator.

Plain numpy, FP64; nothing here is shared with the GPU library, which
implements the same definition in its own kernels.

Definition (the fabricated right-hand sides that stand in for Eqs. 14-16):
  * random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
    random numbers: as easy as 1, 2, 3", SC 2011), key = (seed mod 2^32,
    seed div 2^32), counter = (draw index d, sample s, step mod 2^32,
    step div 2^32); a 32-bit output x maps to u = ((x >> 8) + 1/2) 2^-24;
  * per sample s: draw d = 0 gives the length scale
    l = exp(ln l_lo + u_0 (ln l_hi - ln l_lo));
  * feature f (0 <= f < J): draw d = 1 + f gives, by Box-Muller,
    w = (sqrt(-2 ln u_0) cos(2 pi u_1), sqrt(-2 ln u_0) sin(2 pi u_1)) / l and
    phase phi = 2 pi u_2;
  * Gaussian random field with covariance exp(-|d|^2 / (2 l^2)) by random
    Fourier features (Rahimi & Recht, 2007):
    g(x, y) = sqrt(2 / J) sum_f cos(w_f,x x + w_f,y y + phi_f) at the cell
    centres;
  * R = (cell area) g, minus its mean, divided by its RMS.
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """One Philox4x32 block with 10 rounds; ctr: 4 ints, key: 2 ints (Python ints, exact)."""
    x0, x1, x2, x3 = (int(c) & MASK for c in ctr)
    k0, k1 = (int(k) & MASK for k in key)
    for r in range(10):
        p0 = M0 * x0
        p1 = M1 * x2
        hi0, lo0 = p0 >> 32, p0 & MASK
        hi1, lo1 = p1 >> 32, p1 & MASK
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
        k0 = (k0 + W0) & MASK
        k1 = (k1 + W1) & MASK
    return x0, x1, x2, x3


def philox_vec(d, s, step, seed):
    """Vectorised Philox4x32-10 over arrays of draw indices d (one sample s):
    returns a [len(d), 4] uint64 array of 32-bit outputs."""
    d = np.asarray(d, dtype=np.uint64)
    x0 = d & MASK
    x1 = np.full_like(d, s & MASK)
    x2 = np.full_like(d, step & MASK)
    x3 = np.full_like(d, (step >> 32) & MASK)
    k0, k1 = np.uint64(seed & MASK), np.uint64((seed >> 32) & MASK)
    m = np.uint64(MASK)
    for r in range(10):
        p0 = np.uint64(M0) * x0
        p1 = np.uint64(M1) * x2
        hi0, lo0 = p0 >> np.uint64(32), p0 & m
        hi1, lo1 = p1 >> np.uint64(32), p1 & m
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
        k0 = (k0 + np.uint64(W0)) & m
        k1 = (k1 + np.uint64(W1)) & m
    return np.stack([x0, x1, x2, x3], axis=1)


def to_unit(x):
    """32-bit integers -> uniforms in (0, 1)."""
    return ((np.asarray(x, dtype=np.uint64) >> np.uint64(8)).astype(np.float64) + 0.5) * 2.0 ** -24


def features(s, step, seed, J, len_lo, len_hi):
    """Length scale and (w_x, w_y, phi) of the J features of sample s."""
    u = to_unit(philox_vec(np.arange(J + 1), s, step, seed))
    ell = np.exp(np.log(len_lo) + u[0, 0] * (np.log(len_hi) - np.log(len_lo)))
    rad = np.sqrt(-2.0 * np.log(u[1:, 0]))
    wx = rad * np.cos(2.0 * np.pi * u[1:, 1]) / ell
    wy = rad * np.sin(2.0 * np.pi * u[1:, 1]) / ell
    phi = 2.0 * np.pi * u[1:, 2]
    return ell, wx, wy, phi


def grf_field(xc, yc, wx, wy, phi):
    """g at the cell centres, [ny, nx]."""
    J = len(wx)
    arg = wx[:, None, None] * np.asarray(xc)[None, None, :] + wy[:, None, None] * np.asarray(yc)[None, :, None] \
        + phi[:, None, None]
    return np.sqrt(2.0 / J) * np.cos(arg).sum(axis=0)


GRID_DRAW = 0xFFFFFF00  # counter index of the first grid draw, past the field draws


def grid(nx, ny, seed, step, sample):
    """Grid of fabricated system `sample` at `step`: a tanh-stretched tensor
    grid (stretch factors in [1, 2.5], the range of Table 1's grids) and an
    elliptic obstacle (the immersed bodies of Sec. 3).
      draw GRID_DRAW:     beta_x = 1 + 1.5 u0, beta_y = 1 + 1.5 u1,
                          centre (0.25 + 0.5 u2, 0.25 + 0.5 u3);
      draw GRID_DRAW + 1: semi-axes 0.05 + 0.1 u0, 0.05 + 0.1 u1, angle pi u2;
      faces (1 + tanh(beta (2 i / n - 1)) / tanh beta) / 2, centres at face
      midpoints; a cell is solid when its centre lies in the closed ellipse.
    Returns (xc, yc, hx, hy, mask [ny, nx] uint8, (beta_x, beta_y, cx, cy, a, b, theta))."""
    key = (seed & MASK, (seed >> 32) & MASK)
    d0 = philox4x32_10((GRID_DRAW, sample, step & MASK, (step >> 32) & MASK), key)
    d1 = philox4x32_10((GRID_DRAW + 1, sample, step & MASK, (step >> 32) & MASK), key)
    u0, u1 = to_unit(np.array(d0)), to_unit(np.array(d1))
    bx, by = 1.0 + 1.5 * u0[0], 1.0 + 1.5 * u0[1]
    cx, cy = 0.25 + 0.5 * u0[2], 0.25 + 0.5 * u0[3]
    a, b, th = 0.05 + 0.1 * u1[0], 0.05 + 0.1 * u1[1], np.pi * u1[2]

    def axis(n, beta):
        f = 0.5 * (1.0 + np.tanh(beta * (2.0 * np.arange(n + 1) / n - 1.0)) / np.tanh(beta))
        f[0], f[-1] = 0.0, 1.0
        return 0.5 * (f[1:] + f[:-1]), np.diff(f)

    xc, hx = axis(nx, bx)
    yc, hy = axis(ny, by)
    dx, dy = xc[None, :] - cx, yc[:, None] - cy
    p = (dx * np.cos(th) + dy * np.sin(th)) / a
    q = (dy * np.cos(th) - dx * np.sin(th)) / b
    mask = (p * p + q * q <= 1.0).astype(np.uint8)
    return xc, yc, hx, hy, mask, (bx, by, cx, cy, a, b, th)


def generate(grids, seed, step, J=512, len_lo=0.05, len_hi=0.5):
    """R [nb, ny, nx] for sample s on grids[s] (FP64)."""
    out = []
    for s, g in enumerate(grids):
        _, wx, wy, phi = features(s, step, seed, J, len_lo, len_hi)
        r = grf_field(g.xc, g.yc, wx, wy, phi) * np.outer(g.hy, g.hx)
        r = r - r.mean()
        out.append(r / np.sqrt(np.mean(r * r)))
    return np.stack(out)
