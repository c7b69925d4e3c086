"""Pins of the DeepONet oracle's wiring (CPU only): the whole forward of a tiny
network written out with explicit loops, from the definitions of Sec. 2.4
(Eqs. 17-18 for the Mesh-Conv layer, the branch/trunk combination of the
DeepONet) and the readings the oracle states in its header, compared with
``oracle.net.forward`` to 1e-12.

The grid is not square (8 x 6 cells) and every channel count differs from
the others, so a transposed trunk basis, a swapped concatenation order, a
pooling or upsampling on the wrong axis, or a distance map of the wrong axis
changes the output. The last test plants such mistakes in the oracle (by
monkeypatching its helpers) and checks that the comparison catches each."""
import math

import numpy as np
import pytest
import torch

from paper_2604_01800_amd import inputs
from oracle import net as onet


def tiny_cfg(**kw):
    c = onet.NetConfig(levels=2, base_channels=3, basis=5, trunk_width=4, trunk_hidden=2, phi_hidden=3)
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def tiny_grid(nx=8, ny=6, bx=1.7, by=0.9, seed=11):
    """Stretched grid with a random solid pattern (an ellipse covers too few
    cells of so small a grid to exercise the mask channel)."""
    g = inputs.make_grid(nx, ny, bx, by)
    g.mask = (np.random.default_rng(seed).uniform(size=(ny, nx)) < 0.3).astype(np.uint8)
    return g


def _np_params(p):
    return {k: v.detach().numpy().copy() for k, v in p.items()}


# ---------------------------------------------------------------------------
# The forward written out, one scalar at a time.

def loop_level_geometry(centres, widths, levels):
    """Per level: centres (pairs averaged) and widths (pairs summed)."""
    cs, hs = [list(centres)], [list(widths)]
    for _ in range(1, levels):
        c, h = cs[-1], hs[-1]
        cs.append([(c[2 * i] + c[2 * i + 1]) / 2 for i in range(len(c) // 2)])
        hs.append([h[2 * i] + h[2 * i + 1] for i in range(len(h) // 2)])
    return cs, hs


def loop_distance(c, i, side, scale):
    """Distance from centre i to its left (side -1) or right (+1) neighbour,
    the interior neighbour's distance at a boundary, times scale."""
    n = len(c)
    if side < 0:
        d = c[i] - c[i - 1] if i > 0 else c[1] - c[0]
    else:
        d = c[i + 1] - c[i] if i < n - 1 else c[n - 1] - c[n - 2]
    return d * scale


def loop_mconv(P, name, X, geo, use_eta):
    """conv3x3(eta * X) + b with eta = exp(-Phi(Delta)^2) evaluated at the
    input pixel, one value per node (use_eta = 2) or per input channel
    (use_eta = 1); zero padding. X: [Cin][H][W] lists."""
    cx, cy, sx, sy = geo
    W3, b = P[f"{name}.W"], P[f"{name}.b"]
    W1, b1, W2, b2 = P[f"{name}.phi.W1"], P[f"{name}.phi.b1"], P[f"{name}.phi.W2"], P[f"{name}.phi.b2"]
    cout, cin = W3.shape[0], W3.shape[1]
    H, W = len(X[0]), len(X[0][0])
    eta = [[[1.0] * W for _ in range(H)] for _ in range(cin)]
    if use_eta:
        for j in range(H):
            for i in range(W):
                delta = [loop_distance(cx, i, -1, sx), loop_distance(cx, i, +1, sx),
                         loop_distance(cy, j, -1, sy), loop_distance(cy, j, +1, sy)]
                hid = [math.tanh(sum(W1[a][k] * delta[k] for k in range(4)) + b1[a]) for a in range(len(b1))]
                for c in range(cin):
                    k = 0 if use_eta == 2 else c
                    phi = sum(W2[k][a] * hid[a] for a in range(len(b1))) + b2[k]
                    eta[c][j][i] = math.exp(-phi * phi)
    out = [[[0.0] * W for _ in range(H)] for _ in range(cout)]
    for o in range(cout):
        for j in range(H):
            for i in range(W):
                acc = b[o]
                for c in range(cin):
                    for ky in range(3):
                        for kx in range(3):
                            jj, ii = j + ky - 1, i + kx - 1
                            if 0 <= jj < H and 0 <= ii < W:
                                acc += W3[o][c][ky][kx] * eta[c][jj][ii] * X[c][jj][ii]
                out[o][j][i] = acc
    return out


def relu(X):
    return [[[max(v, 0.0) for v in row] for row in ch] for ch in X]


def loop_forward(P, cfg, g, r, mask):
    N = g.nx * g.ny
    nrm = math.sqrt(sum(float(v) * float(v) for v in r.reshape(-1)))
    rs = [[float(r[j, i]) * math.sqrt(N) / nrm for i in range(g.nx)] for j in range(g.ny)]
    m = [[float(mask[j, i]) for i in range(g.nx)] for j in range(g.ny)]
    Lx, Ly = float(sum(g.hx)), float(sum(g.hy))
    cxs, hxs = loop_level_geometry(list(g.xc), list(g.hx), cfg.levels)
    cys, hys = loop_level_geometry(list(g.yc), list(g.hy), cfg.levels)

    def geo(l):
        return cxs[l], cys[l], len(cxs[l]) / Lx, len(cys[l]) / Ly

    def width_channels(l):
        W, H = len(cxs[l]), len(cys[l])
        sx, sy = W / Lx, H / Ly
        return [[[hxs[l][i] * sx for i in range(W)] for _ in range(H)],
                [[hys[l][j] * sy for _ in range(W)] for j in range(H)]]

    # encoder
    E = []
    for l in range(cfg.levels):
        if l == 0:
            X = [rs, m]
        else:
            prev = E[-1]
            H, W = len(prev[0]) // 2, len(prev[0][0]) // 2
            X = [[[(ch[2 * j][2 * i] + ch[2 * j][2 * i + 1] + ch[2 * j + 1][2 * i] + ch[2 * j + 1][2 * i + 1]) / 4
                   for i in range(W)] for j in range(H)] for ch in prev]
        if cfg.use_spacing:
            X = X + width_channels(l)
        X = relu(loop_mconv(P, f"enc{l}.a", X, geo(l), cfg.use_eta))
        E.append(relu(loop_mconv(P, f"enc{l}.b", X, geo(l), cfg.use_eta)))
    # decoder: 1x1 up-conv of the coarser result, nearest 2x upsampling, then
    # concatenation in the order [upsampled, encoder skip, widths]
    d = E[-1]
    for l in range(cfg.levels - 2, -1, -1):
        Wu, bu = P[f"up{l}.W"], P[f"up{l}.b"]
        Hc, Wc = len(d[0]), len(d[0][0])
        u = [[[bu[o] + sum(Wu[o][c] * d[c][j][i] for c in range(len(d))) for i in range(Wc)] for j in range(Hc)]
             for o in range(len(bu))]
        up = [[[ch[j // 2][i // 2] for i in range(2 * Wc)] for j in range(2 * Hc)] for ch in u]
        X = up + E[l] + (width_channels(l) if cfg.use_spacing else [])
        X = relu(loop_mconv(P, f"dec{l}.c", X, geo(l), cfg.use_eta))
        d = relu(loop_mconv(P, f"dec{l}.d", X, geo(l), cfg.use_eta))
    # head: branch coefficients B_k at every pixel
    Wh, bh = P["head.W"], P["head.b"]
    # trunk at the pixel's normalised centre coordinates (x along i, y along j)
    x0, y0 = g.xc[0] - g.hx[0] / 2, g.yc[0] - g.hy[0] / 2
    y = np.zeros((g.ny, g.nx))
    for j in range(g.ny):
        for i in range(g.nx):
            t = [2 * (g.xc[i] - x0) / Lx - 1, 2 * (g.yc[j] - y0) / Ly - 1]
            for k in range(cfg.trunk_hidden):
                Wt, bt = P[f"trunk{k}.W"], P[f"trunk{k}.b"]
                t = [math.tanh(bt[a] + sum(Wt[a][c] * t[c] for c in range(len(t)))) for a in range(len(bt))]
            Wo, bo = P["trunk_out.W"], P["trunk_out.b"]
            T = [bo[k] + sum(Wo[k][c] * t[c] for c in range(len(t))) for k in range(cfg.basis)]
            B = [bh[k] + sum(Wh[k][c] * d[c][j][i] for c in range(len(d))) for k in range(cfg.basis)]
            y[j, i] = P["gamma"][0] * sum(B[k] * T[k] for k in range(cfg.basis))
    return y


# ---------------------------------------------------------------------------

@pytest.mark.parametrize("use_eta,use_spacing", [(2, 1), (1, 1), (0, 1), (2, 0)])
def test_forward_matches_explicit_loops(use_eta, use_spacing):
    cfg = tiny_cfg(use_eta=use_eta, use_spacing=use_spacing)
    g = tiny_grid()
    assert g.mask.any() and not g.mask.all()
    p = onet.init_params(cfg, np.random.default_rng(5), phi_scale=1.0)
    r = np.random.default_rng(6).standard_normal((g.ny, g.nx))
    y = onet.forward(p, cfg, g, r[None], g.mask)[0].numpy()
    ref = loop_forward(_np_params(p), cfg, g, r, g.mask)
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_three_level_forward_matches_explicit_loops():
    cfg = tiny_cfg(levels=3, base_channels=2)
    g = tiny_grid(8, 12, 1.3, 2.2, seed=2)
    p = onet.init_params(cfg, np.random.default_rng(8), phi_scale=1.0)
    r = np.random.default_rng(9).standard_normal((g.ny, g.nx))
    y = onet.forward(p, cfg, g, r[None], g.mask)[0].numpy()
    ref = loop_forward(_np_params(p), cfg, g, r, g.mask)
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("use_eta", [2, 1])
def test_planted_wiring_mistakes_are_caught(monkeypatch, use_eta):
    """Each planted mistake in the oracle moves its output away from the
    explicit loops by far more than rounding (the loops agree with the
    oracle to 1e-12; every mistake moves it by more than 1e-5)."""
    cfg = tiny_cfg(use_eta=use_eta)
    g = tiny_grid()
    p = onet.init_params(cfg, np.random.default_rng(5), phi_scale=1.0)
    r = np.random.default_rng(6).standard_normal((g.ny, g.nx))
    ref = loop_forward(_np_params(p), cfg, g, r, g.mask)

    def rel_err():
        y = onet.forward(p, cfg, g, r[None], g.mask)[0].numpy()
        return np.linalg.norm(y - ref) / np.linalg.norm(ref)

    assert rel_err() <= 1e-12
    real_trunk_input, real_cat, real_features = onet.trunk_input, torch.cat, onet.grid_features

    # 1. trunk basis transposed: (y, x) fed where (x, y) belongs
    monkeypatch.setattr(onet, "trunk_input", lambda grid: real_trunk_input(grid).flip(1))
    assert rel_err() > 1e-5
    monkeypatch.setattr(onet, "trunk_input", real_trunk_input)

    # 2. decoder concatenation in the order [skip, upsampled, widths]
    def swapped_cat(parts, dim=0):
        if dim == 1 and len(parts) == 3 and parts[0].shape[1] == parts[1].shape[1] == cfg.base_channels:
            parts = [parts[1], parts[0], parts[2]]
        return real_cat(parts, dim=dim)

    monkeypatch.setattr(onet.torch, "cat", swapped_cat)
    assert rel_err() > 1e-5
    monkeypatch.setattr(onet.torch, "cat", real_cat)

    # 3. distance maps of the two axes exchanged (left/right <-> down/up)
    def swapped_axes(grid, c):
        return [(d[[2, 3, 0, 1]].contiguous(), w) for d, w in real_features(grid, c)]

    monkeypatch.setattr(onet, "grid_features", swapped_axes)
    assert rel_err() > 1e-5
    monkeypatch.setattr(onet, "grid_features", real_features)
    assert rel_err() <= 1e-12
