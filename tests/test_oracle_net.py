"""Pins of the FP64 DeepONet / Mesh-Conv oracle (CPU only)."""
import math

import numpy as np
import pytest
import torch

from paper_2604_01800_amd import inputs
from oracle import direct
from oracle import net as onet


def small_cfg(**kw):
    c = onet.NetConfig(levels=3, base_channels=4, basis=6, trunk_width=8, trunk_hidden=2, phi_hidden=3)
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def test_param_count_default():
    cfg = onet.NetConfig()
    n = onet.num_params(cfg)
    # conv weights ~1.8 M for 32/64/128/256 channels, trunk ~66 K
    assert 1.7e6 < n < 2.1e6, n


@pytest.mark.parametrize("per_node", [False, True])
def test_mconv_matches_explicit_loops(per_node):
    """Eqs. 17-18 written out: one local weight per node (use_eta = 2) or one
    per input channel (use_eta = 1)."""
    rng = np.random.default_rng(0)
    cin, cout, H, W, Hd = 3, 2, 5, 6, 3
    k = 1 if per_node else cin
    p = {"m.W": torch.from_numpy(rng.standard_normal((cout, cin, 3, 3))),
         "m.b": torch.from_numpy(rng.standard_normal(cout)),
         "m.phi.W1": torch.from_numpy(rng.standard_normal((Hd, 4))),
         "m.phi.b1": torch.from_numpy(rng.standard_normal(Hd)),
         "m.phi.W2": torch.from_numpy(rng.standard_normal((k, Hd))),
         "m.phi.b2": torch.from_numpy(rng.standard_normal(k))}
    X = rng.standard_normal((1, cin, H, W))
    delta = rng.uniform(0.2, 2.0, size=(4, H, W))
    Y = onet.mconv(p, "m", torch.from_numpy(X), torch.from_numpy(delta), 2 if per_node else 1).numpy()
    W1, b1, W2, b2 = (p[k].numpy() for k in ("m.phi.W1", "m.phi.b1", "m.phi.W2", "m.phi.b2"))
    Wc, bc = p["m.W"].numpy(), p["m.b"].numpy()
    ref = np.zeros((1, cout, H, W))
    for y in range(H):
        for x in range(W):
            for co in range(cout):
                acc = bc[co]
                for ky in range(3):
                    for kx in range(3):
                        yy, xx = y + ky - 1, x + kx - 1
                        if not (0 <= yy < H and 0 <= xx < W):
                            continue
                        h = [math.tanh(sum(W1[a, k] * delta[k, yy, xx] for k in range(4)) + b1[a]) for a in range(Hd)]
                        for ci in range(cin):
                            kk = 0 if per_node else ci
                            phi = sum(W2[kk, a] * h[a] for a in range(Hd)) + b2[kk]
                            acc += Wc[co, ci, ky, kx] * math.exp(-phi * phi) * X[0, ci, yy, xx]
                ref[0, co, y, x] = acc
    np.testing.assert_allclose(Y, ref, rtol=1e-12, atol=1e-12)


def test_uniform_grid_eta_is_constant():
    cfg = small_cfg()
    g = inputs.make_grid(16, 24, 0.0)
    feats = onet.grid_features(g, cfg)
    rng = np.random.default_rng(1)
    p = onet.init_params(cfg, rng)
    for l, (delta, widths) in enumerate(feats):
        eta = onet.eta_map(p, f"enc{l}.b", delta, 1)
        assert torch.allclose(eta, eta[:, :1, :1].expand_as(eta), atol=1e-12)
        # unit spacing everywhere after normalisation by the mean spacing
        assert torch.allclose(delta, torch.ones_like(delta), atol=1e-12)
        assert torch.allclose(widths, torch.ones_like(widths), atol=1e-12)


def test_level_coordinates_closed_form():
    n, beta, L = 64, 2.0, 4
    faces = inputs.tanh_faces(n, beta)
    g = inputs.make_grid(n, n, beta)
    cs, hs = onet.level_coords(g.xc, g.hx, L)
    for l in range(L):
        k = 2 ** l
        np.testing.assert_allclose(hs[l], faces[k::k] - faces[:-k:k][: n // k], rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(cs[l], np.mean(g.xc.reshape(-1, k), axis=1), rtol=1e-13)


def test_boundary_padding_nearest_neighbour():
    g = inputs.make_grid(32, 16, 1.5, 2.5)
    cfg = small_cfg()
    feats = onet.grid_features(g, cfg)
    for delta, _ in feats:
        d = delta.numpy()
        assert np.allclose(d[0, :, 0], d[0, :, 1]) and np.allclose(d[1, :, -1], d[1, :, -2])
        assert np.allclose(d[2, 0, :], d[2, 1, :]) and np.allclose(d[3, -1, :], d[3, -2, :])
        assert np.allclose(d[1, :, :-1], d[0, :, 1:])  # right distance of i = left distance of i+1


def test_input_scale_invariance():
    cfg = small_cfg()
    g = inputs.make_grid(16, 16, 1.5)
    p = onet.init_params(cfg, np.random.default_rng(2))
    r = np.random.default_rng(3).standard_normal((16, 16))
    y1 = onet.forward(p, cfg, g, r)
    y2 = onet.forward(p, cfg, g, 37.5 * r)
    torch.testing.assert_close(y1, y2, rtol=1e-12, atol=1e-12)


def test_branch_translation_equivariance():
    # On a uniform grid (constant eta and widths) the branch commutes with
    # shifts by multiples of 2^(L-1), away from the borders.
    cfg = small_cfg()
    n, s = 96, 8
    g = inputs.make_grid(n, n, 0.0)
    feats = onet.grid_features(g, cfg)
    p = onet.init_params(cfg, np.random.default_rng(4))
    x = torch.zeros((1, 2, n, n), dtype=torch.float64)
    x[0, 0, 36:60, 36:60] = torch.from_numpy(np.random.default_rng(5).standard_normal((24, 24)))
    xs = torch.roll(x, shifts=(s, s), dims=(2, 3))
    b1 = onet.branch(p, cfg, x, feats)
    b2 = onet.branch(p, cfg, xs, feats)
    # the receptive-field radius of this 3-level U-Net is about 23 pixels, so
    # the compared windows stay at least 24 pixels from every border
    torch.testing.assert_close(b2[..., 32 + s:64 + s, 32 + s:64 + s], b1[..., 32:64, 32:64], rtol=1e-10, atol=1e-10)


def test_conv_ablation_flag():
    cfg = small_cfg(use_eta=0)
    g = inputs.make_grid(16, 16, 2.0)
    feats = onet.grid_features(g, cfg)
    p = onet.init_params(cfg, np.random.default_rng(6))
    eta = onet.eta_map(p, "enc0.a", feats[0][0], 0)
    assert torch.all(eta == 1)


def _apply_torch(g):
    """Differentiable FP64 operator (the Kronecker form, built independently)."""
    from oracle import direct
    A = torch.from_numpy(direct.kron_matrix(g))
    return lambda grid, y: (A @ y.reshape(-1)).reshape(y.shape)


def test_fd_gradients_of_residual_loss():
    cfg = small_cfg()
    n = 16
    rng = np.random.default_rng(7)
    grids = [inputs.make_grid(n, n, b) for b in (1.2, 2.1)]
    R = np.stack([inputs.grf(gr, 10 + i, ell=0.2, J=64) for i, gr in enumerate(grids)])
    R -= R.mean(axis=(1, 2), keepdims=True)
    p = onet.init_params(cfg, rng)
    for t in p.values():
        t.requires_grad_(True)
    apply = _apply_torch(grids[0])
    applies = {id(gr): _apply_torch(gr) for gr in grids}
    app = lambda grid, y: applies[id(grid)](grid, y)
    loss = onet.residual_loss(p, cfg, grids, R, apply=app)
    loss.backward()
    names = ["enc0.a.W", "enc1.b.phi.W2", "dec0.c.phi.W1", "up1.W", "head.b", "trunk0.W", "trunk_out.W",
             "gamma", "enc2.a.b", "dec1.d.W"]
    checked = 0
    for name in names:
        t = p[name]
        flat = t.detach().reshape(-1)
        for idx in rng.choice(flat.numel(), size=min(3, flat.numel()), replace=False):
            v0 = float(flat[idx])
            h = 1e-6 * max(1.0, abs(v0))
            vals = []
            for sgn in (+1, -1):
                with torch.no_grad():
                    q = {k: v.detach().clone() for k, v in p.items()}
                    q[name].reshape(-1)[idx] = v0 + sgn * h
                    vals.append(float(onet.residual_loss(q, cfg, grids, R, apply=app)))
            fd = (vals[0] - vals[1]) / (2 * h)
            an = float(t.grad.reshape(-1)[idx])
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * abs(float(loss.detach()))), (name, idx, fd, an)
            checked += 1
    assert checked >= 20


def test_bf16_round_known_values_and_ties():
    """The oracle's BF16 rounding: exact values stay, halfway cases go to the
    even neighbour, anything past halfway rounds away from zero, carries
    reach the exponent; and it agrees with torch's float32 -> bfloat16
    conversion (round to nearest even) on random values of every magnitude."""
    u = 2.0 ** -7  # spacing of bfloat16 values in [1, 2)
    cases = [(1.0, 1.0), (1.0 + u, 1.0 + u), (1.0 + u / 2, 1.0), (1.0 + 3 * u / 2, 1.0 + 2 * u),
             (1.0 + u / 2 + 2.0 ** -20, 1.0 + u), (1.0 + u / 2 - 2.0 ** -20, 1.0),
             (-(1.0 + 3 * u / 2), -(1.0 + 2 * u)), (2.0 - u / 2, 2.0), (0.0, 0.0), (-0.0, -0.0),
             (3.0 * 2.0 ** -130, 3.0 * 2.0 ** -130)]
    x = np.array([c[0] for c in cases], dtype=np.float32)
    want = np.array([c[1] for c in cases], dtype=np.float32)
    got = onet.bf16_round(x)
    np.testing.assert_array_equal(got.view(np.uint32), want.view(np.uint32))
    rng = np.random.default_rng(0)
    v = (rng.standard_normal(200000) * np.exp(rng.uniform(-60, 60, 200000))).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(onet.bf16_round(v).view(np.uint32), ref.view(np.uint32))


def test_sam_gradient_definition():
    """The oracle's SAM gradient equals the plain gradient taken at the
    explicitly perturbed parameters w + rho g / |g| (whole-vector norm), and
    reduces to the plain gradient at rho = 0."""
    cfg = small_cfg()
    g = inputs.make_grid(16, 16, 1.4)
    R = inputs.grf(g, 3, ell=0.2, J=64)[None]
    R = R - R.mean()
    from oracle import direct
    A = torch.from_numpy(direct.kron_matrix(g))
    app = lambda grid, y: (A @ y.reshape(-1)).reshape(y.shape)
    p = onet.init_params(cfg, np.random.default_rng(2))
    l0, g0 = onet.loss_and_grad(p, cfg, [g], R, apply=app)
    ls, gs = onet.sam_gradient(p, cfg, [g], R, 0.0, apply=app, bf16=False)
    assert ls == l0 and all(torch.equal(gs[k], g0[k]) for k in g0)
    flat = onet.flatten(cfg, g0)
    rho = 0.03
    w = onet.unflatten(cfg, onet.flatten(cfg, p) + rho * flat / np.linalg.norm(flat))
    lw, gw = onet.loss_and_grad(w, cfg, [g], R, apply=app)
    ls, gs = onet.sam_gradient(p, cfg, [g], R, rho, apply=app, bf16=False)
    assert abs(ls - lw) <= 1e-12 * lw
    np.testing.assert_allclose(onet.flatten(cfg, gs), onet.flatten(cfg, gw), rtol=1e-10, atol=1e-12)
    assert ls > l0  # the step along +g/|g| climbs the loss


def test_supervised_loss_invariances():
    """The supervised misfit is 0 for any y = c e + d (c != 0), 1 for a y
    orthogonal to the centred target, lies in [0, 1], and is unchanged by
    scaling or shifting either field."""
    rng = np.random.default_rng(3)
    e = torch.from_numpy(rng.standard_normal((12, 10)))
    y = torch.from_numpy(rng.standard_normal((12, 10)))
    f = onet.supervised_loss_of
    assert abs(float(f(-2.5 * e + 7.0, e))) <= 1e-14
    e0 = e - e.mean()
    y0 = y - y.mean()
    orth = y0 - (y0 * e0).sum() / (e0 * e0).sum() * e0
    assert abs(float(f(orth, e)) - 1.0) <= 1e-14
    v = float(f(y, e))
    assert 0.0 < v < 1.0
    for c, d in [(3.0, 0.0), (-0.1, 5.0), (1e4, -2.0)]:
        assert abs(float(f(c * y + d, e)) - v) <= 1e-12
        assert abs(float(f(y, c * e + d)) - v) <= 1e-12


def test_fd_gradients_of_supervised_loss():
    cfg = small_cfg()
    n = 16
    rng = np.random.default_rng(8)
    grids = [inputs.make_grid(n, n, b) for b in (1.3, 2.0)]
    R = np.stack([inputs.grf(gr, 20 + i, ell=0.2, J=64) for i, gr in enumerate(grids)])
    R -= R.mean(axis=(1, 2), keepdims=True)
    T = rng.standard_normal(R.shape)
    p = onet.init_params(cfg, rng)
    for t in p.values():
        t.requires_grad_(True)
    loss = onet.supervised_loss(p, cfg, grids, R, T)
    loss.backward()
    checked = 0
    for name in ["enc0.a.W", "dec0.d.W", "head.W", "trunk1.W", "gamma", "enc1.b.phi.W1", "up0.b"]:
        t = p[name]
        flat = t.detach().reshape(-1)
        for idx in rng.choice(flat.numel(), size=min(3, flat.numel()), replace=False):
            v0 = float(flat[idx])
            h = 1e-6 * max(1.0, abs(v0))
            vals = []
            for sgn in (+1, -1):
                with torch.no_grad():
                    q = {k: v.detach().clone() for k, v in p.items()}
                    q[name].reshape(-1)[idx] = v0 + sgn * h
                    vals.append(float(onet.supervised_loss(q, cfg, grids, R, T)))
            fd = (vals[0] - vals[1]) / (2 * h)
            an = float(t.grad.reshape(-1)[idx])
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * abs(float(loss.detach()))), (name, idx, fd, an)
            checked += 1
    assert checked >= 15


def test_anorm_loss_is_the_line_search_share(orc):
    """The A-norm loss equals |e - alpha y|_A^2 / |e|_A^2 after the exact
    line search alpha = (R . y) / (y . A y) along y (Eqs. 12-13), computed
    here from the error directly; it is 0 for y = c e + d and 1 for a y
    A-orthogonal to e."""
    g = inputs.make_grid(14, 11, 1.7, 1.2)
    rng = np.random.default_rng(12)
    e = rng.standard_normal((11, 14))
    e -= e.mean()
    R = orc.apply(g, e)
    y = rng.standard_normal((11, 14))
    A = lambda v: orc.apply(g, v)
    alpha = (R * y).sum() / (y * A(y)).sum()
    d = e - alpha * y
    want = (d * A(d)).sum() / (e * A(e)).sum()
    t = lambda a: torch.from_numpy(np.asarray(a, dtype=np.float64))
    got = float(onet.anorm_loss_of(t(y), t(R), t(e), t(A(y))))
    assert abs(got - want) <= 1e-13
    assert 0.0 < got < 1.0
    for c, dd in [(-2.5, 0.0), (0.3, 4.0)]:
        yy = c * e + dd
        assert abs(float(onet.anorm_loss_of(t(yy), t(R), t(e), t(A(yy))))) <= 1e-13
    # a direction A-orthogonal to e removes nothing
    z = y - (y * A(e)).sum() / (e * A(e)).sum() * e
    assert abs(float(onet.anorm_loss_of(t(z), t(R), t(e), t(A(z)))) - 1.0) <= 1e-13


def test_anorm_loss_on_two_eigenmodes(orc):
    """Uniform grid: with e = v1 + v2 (cosine eigenvectors of A with
    eigenvalues l1, l2) and y = v1 the loss is l2|v2|^2 / (l1|v1|^2 + l2|v2|^2)."""
    n = 12
    g = inputs.make_grid(n, n, 0.0)
    h = 1.0 / n
    xc = (np.arange(n) + 0.5) * h
    v1 = np.outer(np.ones(n), np.cos(np.pi * xc))
    v2 = np.outer(np.cos(3 * np.pi * xc), np.cos(2 * np.pi * xc))
    lam = lambda kx, ky: (2 - 2 * np.cos(np.pi * kx * h)) / h ** 2 * h * h + (2 - 2 * np.cos(np.pi * ky * h)) / h ** 2 * h * h
    l1, l2 = lam(1, 0), lam(2, 3)
    np.testing.assert_allclose(orc.apply(g, v1), l1 * v1, atol=1e-12)
    np.testing.assert_allclose(orc.apply(g, v2), l2 * v2, atol=1e-12)
    e = v1 + v2
    R = orc.apply(g, e)
    t = lambda a: torch.from_numpy(np.asarray(a, dtype=np.float64))
    got = float(onet.anorm_loss_of(t(v1), t(R), t(e), t(orc.apply(g, v1))))
    n1, n2 = (v1 * v1).sum(), (v2 * v2).sum()
    assert abs(got - l2 * n2 / (l1 * n1 + l2 * n2)) <= 1e-12


def test_fd_gradients_of_anorm_loss(orc):
    cfg = small_cfg()
    n = 16
    rng = np.random.default_rng(9)
    grids = [inputs.make_grid(n, n, b) for b in (1.3, 2.0)]
    E = rng.standard_normal((2, n, n))
    R = np.stack([orc.apply(gr, E[i]) for i, gr in enumerate(grids)])
    mats = {id(gr): torch.from_numpy(direct.kron_matrix(gr)) for gr in grids}
    app = lambda gr, y: (mats[id(gr)] @ y.reshape(-1)).reshape(y.shape)
    p = onet.init_params(cfg, rng)
    for t in p.values():
        t.requires_grad_(True)
    loss = onet.anorm_loss(p, cfg, grids, R, E, apply=app)
    loss.backward()
    checked = 0
    for name in ["enc0.a.W", "dec0.d.W", "head.W", "trunk1.W", "enc1.b.phi.W1", "up0.b"]:
        t = p[name]
        flat = t.detach().reshape(-1)
        for idx in rng.choice(flat.numel(), size=min(3, flat.numel()), replace=False):
            v0 = float(flat[idx])
            h = 1e-6 * max(1.0, abs(v0))
            vals = []
            for sgn in (+1, -1):
                with torch.no_grad():
                    q = {k: v.detach().clone() for k, v in p.items()}
                    q[name].reshape(-1)[idx] = v0 + sgn * h
                    vals.append(float(onet.anorm_loss(q, cfg, grids, R, E, apply=app)))
            fd = (vals[0] - vals[1]) / (2 * h)
            an = float(t.grad.reshape(-1)[idx])
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * abs(float(loss.detach()))), (name, idx, fd, an)
            checked += 1
    assert checked >= 12


def test_per_node_weight_is_the_per_channel_form_with_equal_rows():
    """use_eta = 2 (one local weight per node) gives the forward of use_eta = 1
    whose Phi output rows are all equal to the single row, and its Phi output
    gradient is the sum of the per-channel rows' gradients."""
    cfg2 = small_cfg(use_eta=2)
    cfg1 = small_cfg(use_eta=1)
    rng = np.random.default_rng(21)
    p2 = onet.init_params(cfg2, rng, phi_scale=1.0)
    p1 = {}
    for name, shape in onet.param_spec(cfg1):
        t = p2[name]
        p1[name] = t.expand(shape).clone() if (".phi.W2" in name or ".phi.b2" in name) else t.clone()
    g = inputs.make_grid(16, 12, 1.7, 1.2)
    g.mask = np.zeros((12, 16), np.uint8)
    R = inputs.grf(g, 3, ell=0.2, J=64)[None]
    for t in list(p1.values()) + list(p2.values()):
        t.requires_grad_(True)
    y1 = onet.forward(p1, cfg1, g, R, g.mask)
    y2 = onet.forward(p2, cfg2, g, R, g.mask)
    np.testing.assert_allclose(y1.detach().numpy(), y2.detach().numpy(), rtol=1e-13, atol=1e-13)
    w = torch.from_numpy(np.random.default_rng(5).standard_normal(y1.shape))
    (y1 * w).sum().backward()
    (y2 * w).sum().backward()
    for name in ("enc0.a.phi.W2", "dec1.c.phi.b2", "enc2.b.phi.W2"):
        np.testing.assert_allclose(p1[name].grad.sum(0).numpy(), p2[name].grad[0].numpy(), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(p1["enc1.a.phi.W1"].grad.numpy(), p2["enc1.a.phi.W1"].grad.numpy(), rtol=1e-11,
                               atol=1e-13)


def test_fd_gradients_per_node_weights():
    cfg = small_cfg(use_eta=2)
    n = 16
    rng = np.random.default_rng(17)
    grids = [inputs.make_grid(n, n, b) for b in (1.4, 1.9)]
    R = np.stack([inputs.grf(gr, 30 + i, ell=0.2, J=64) for i, gr in enumerate(grids)])
    R -= R.mean(axis=(1, 2), keepdims=True)
    p = onet.init_params(cfg, rng, phi_scale=1.0)
    for t in p.values():
        t.requires_grad_(True)
    applies = {id(gr): _apply_torch(gr) for gr in grids}
    app = lambda grid, y: applies[id(grid)](grid, y)
    loss = onet.residual_loss(p, cfg, grids, R, apply=app)
    loss.backward()
    checked = 0
    for name in ["enc0.a.phi.W2", "enc1.b.phi.b2", "dec0.c.phi.W1", "dec1.d.phi.W2", "enc0.b.W"]:
        t = p[name]
        flat = t.detach().reshape(-1)
        for idx in rng.choice(flat.numel(), size=min(3, flat.numel()), replace=False):
            v0 = float(flat[idx])
            h = 1e-6 * max(1.0, abs(v0))
            vals = []
            for sgn in (+1, -1):
                with torch.no_grad():
                    q = {k: v.detach().clone() for k, v in p.items()}
                    q[name].reshape(-1)[idx] = v0 + sgn * h
                    vals.append(float(onet.residual_loss(q, cfg, grids, R, apply=app)))
            fd = (vals[0] - vals[1]) / (2 * h)
            an = float(t.grad.reshape(-1)[idx])
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * abs(float(loss.detach()))), (name, idx, fd, an)
            checked += 1
    assert checked >= 10
