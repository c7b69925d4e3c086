"""TEST INFRASTRUCTURE — FP64 reference of the DeepONet used by the line search.

Plain PyTorch CPU float64 (library conv2d / pooling / interpolation as steps,
autograd for gradients); nothing here is shared with the GPU library.

Architecture (Sec. 2.4; the figures are not available, so the concrete
choices below are this implementation's reading, stated once here):

* Mesh-Conv layer (Eqs. 17-18): per pixel, the distance vector Delta holds the
  distances to the four orthogonal neighbours (left, right, down, up) at the
  layer's resolution; a small network Phi (4 -> hidden, tanh -> K) maps it to
  the local weight eta = exp(-Phi^2); the layer computes conv3x3(eta * X) +
  bias (zero padding). use_eta = 2: K = 1, one weight per node multiplying
  the whole feature vector, as Eqs. 17-18 are written; use_eta = 1: K = C_in,
  one weight per input channel (a generalisation); use_eta = 0: a standard
  convolution (the paper's "-Conv" variant).
* Multi-level distance maps: the cell-centre coordinates are average-pooled
  level by level (pairs of centres), distances are taken between pooled
  centres, the exterior distance at a boundary pixel equals its interior
  neighbour distance (nearest-neighbour padding), and distances are divided
  by the level's mean spacing (domain length / pixels).
* Branch: a U-Net with L levels and C_l = C * 2^l channels. Encoder level l:
  input = (l == 0 ? [scaled residual, mask] : avgpool2(E_{l-1})) followed by
  the two normalised width channels (hx, hy) of the level; two Mesh-Conv +
  ReLU layers give E_l. Decoder level l (L-2 .. 0): nearest 2x upsampling of
  a 1x1 conv (C_{l+1} -> C_l) of D_{l+1} (D_{L-1} = E_{L-1}), concatenated with
  E_l and the two width channels; two Mesh-Conv + ReLU layers give D_l. Head:
  1x1 conv C_0 -> P giving the branch coefficients B(p) at every pixel.
* Trunk: MLP on the normalised cell-centre coordinates in [-1, 1]^2, tanh
  hidden layers, linear output of P basis values T(p).
* Output: y(p) = gamma * sum_k B_k(p) T_k(p).
* Input scaling: the residual is scaled to unit RMS, r * sqrt(N) / ||r||.

The flat parameter vector lists, in order: for each encoder level l = 0..L-1
the layers (a, b); for each decoder level l = L-2..0 the 1x1 up-conv then the
layers (c, d); the head; the trunk layers; gamma. A Mesh-Conv layer holds
W [Cout, Cin, 3, 3], b [Cout], phi.W1 [H, 4], phi.b1 [H], phi.W2 [K, H],
phi.b2 [K] (K = 1 with use_eta = 2, else Cin). A 1x1 conv holds W [Cout, Cin], b [Cout]. A trunk layer holds
W [out, in], b [out].
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch
import torch.nn.functional as F


@dataclasses.dataclass
class NetConfig:
    levels: int = 4
    base_channels: int = 32
    in_channels: int = 2  # scaled residual, mask
    basis: int = 128
    trunk_width: int = 128
    trunk_hidden: int = 4
    phi_hidden: int = 16
    use_eta: int = 2
    use_spacing: int = 1

    def ch(self, l):
        return self.base_channels << l


def _mconv_spec(name, cin, cout, H, per_node=False):
    k = 1 if per_node else cin
    return [(f"{name}.W", (cout, cin, 3, 3)), (f"{name}.b", (cout,)),
            (f"{name}.phi.W1", (H, 4)), (f"{name}.phi.b1", (H,)),
            (f"{name}.phi.W2", (k, H)), (f"{name}.phi.b2", (k,))]


def param_spec(cfg: NetConfig):
    """Ordered (name, shape) list of the flat parameter vector."""
    L, H, sp, pn = cfg.levels, cfg.phi_hidden, 2 * cfg.use_spacing, cfg.use_eta == 2
    spec = []
    for l in range(L):
        cin = (cfg.in_channels if l == 0 else cfg.ch(l - 1)) + sp
        spec += _mconv_spec(f"enc{l}.a", cin, cfg.ch(l), H, pn)
        spec += _mconv_spec(f"enc{l}.b", cfg.ch(l), cfg.ch(l), H, pn)
    for l in range(L - 2, -1, -1):
        spec += [(f"up{l}.W", (cfg.ch(l), cfg.ch(l + 1))), (f"up{l}.b", (cfg.ch(l),))]
        spec += _mconv_spec(f"dec{l}.c", 2 * cfg.ch(l) + sp, cfg.ch(l), H, pn)
        spec += _mconv_spec(f"dec{l}.d", cfg.ch(l), cfg.ch(l), H, pn)
    spec += [("head.W", (cfg.basis, cfg.ch(0))), ("head.b", (cfg.basis,))]
    w, nin = cfg.trunk_width, 2
    for k in range(cfg.trunk_hidden):
        spec += [(f"trunk{k}.W", (w, nin)), (f"trunk{k}.b", (w,))]
        nin = w
    spec += [("trunk_out.W", (cfg.basis, nin)), ("trunk_out.b", (cfg.basis,)), ("gamma", (1,))]
    return spec


def num_params(cfg: NetConfig) -> int:
    return sum(int(np.prod(s)) for _, s in param_spec(cfg))


def bf16_params(cfg: NetConfig):
    """Names of the parameters the GPU consumes in BF16 (matrix operands)."""
    out = set()
    for name, shape in param_spec(cfg):
        if name.endswith(".W") and ".phi." not in name:
            out.add(name)
    return out


def unflatten(cfg: NetConfig, flat):
    flat = torch.as_tensor(np.asarray(flat, dtype=np.float64))
    out, k = {}, 0
    for name, shape in param_spec(cfg):
        n = int(np.prod(shape))
        out[name] = flat[k:k + n].reshape(shape).clone()
        k += n
    assert k == flat.numel(), (k, flat.numel())
    return out


def flatten(cfg: NetConfig, params) -> np.ndarray:
    return np.concatenate([params[n].detach().reshape(-1).numpy() for n, _ in param_spec(cfg)])


# ---------------------------------------------------------------------------
# Grid-derived inputs (per level).

def level_coords(xc, hx, levels):
    """Average-pooled centres and merged widths for levels 0..levels-1."""
    cs, hs = [np.asarray(xc, np.float64)], [np.asarray(hx, np.float64)]
    for _ in range(1, levels):
        c, h = cs[-1], hs[-1]
        cs.append(0.5 * (c[0::2] + c[1::2]))
        hs.append(h[0::2] + h[1::2])
    return cs, hs


def neighbour_distances(c):
    """(left, right) distances with nearest-neighbour padding at both ends."""
    d = np.diff(c)
    left = np.concatenate([[d[0]], d])
    right = np.concatenate([d, [d[-1]]])
    return left, right


def grid_features(grid, cfg: NetConfig):
    """Per level: Delta [4, H, W] (left, right, down, up) and widths [2, H, W],
    both normalised by the level's mean spacing."""
    Lx, Ly = float(np.sum(grid.hx)), float(np.sum(grid.hy))
    cx, hxs = level_coords(grid.xc, grid.hx, cfg.levels)
    cy, hys = level_coords(grid.yc, grid.hy, cfg.levels)
    feats = []
    for l in range(cfg.levels):
        W, H = len(cx[l]), len(cy[l])
        sx, sy = W / Lx, H / Ly
        xl, xr = neighbour_distances(cx[l])
        yd, yu = neighbour_distances(cy[l])
        delta = np.stack([np.broadcast_to(xl * sx, (H, W)), np.broadcast_to(xr * sx, (H, W)),
                          np.broadcast_to((yd * sy)[:, None], (H, W)), np.broadcast_to((yu * sy)[:, None], (H, W))])
        widths = np.stack([np.broadcast_to(hxs[l] * sx, (H, W)), np.broadcast_to((hys[l] * sy)[:, None], (H, W))])
        feats.append((torch.from_numpy(np.ascontiguousarray(delta)), torch.from_numpy(np.ascontiguousarray(widths))))
    return feats


def trunk_input(grid):
    Lx, Ly = float(np.sum(grid.hx)), float(np.sum(grid.hy))
    x0 = grid.xc[0] - 0.5 * grid.hx[0]
    y0 = grid.yc[0] - 0.5 * grid.hy[0]
    xs = 2.0 * (np.asarray(grid.xc) - x0) / Lx - 1.0
    ys = 2.0 * (np.asarray(grid.yc) - y0) / Ly - 1.0
    X = np.broadcast_to(xs[None, :], (grid.ny, grid.nx))
    Y = np.broadcast_to(ys[:, None], (grid.ny, grid.nx))
    return torch.from_numpy(np.stack([X, Y], axis=-1).reshape(-1, 2).copy())


# ---------------------------------------------------------------------------
# Layers.

def eta_map(p, name, delta, use_eta):
    """Local weight of Eq. 17: [K, H, W] (K = 1 per node, or one per input
    channel), broadcast over the channels when K = 1."""
    cin = p[f"{name}.phi.W2"].shape[0]
    if not use_eta:
        return torch.ones((cin,) + tuple(delta.shape[1:]), dtype=torch.float64)
    d = delta.reshape(4, -1).T  # [HW, 4]
    h = torch.tanh(d @ p[f"{name}.phi.W1"].T + p[f"{name}.phi.b1"])
    phi = h @ p[f"{name}.phi.W2"].T + p[f"{name}.phi.b2"]  # [HW, Cin]
    return torch.exp(-phi * phi).T.reshape((cin,) + tuple(delta.shape[1:]))


def mconv(p, name, X, delta, use_eta):
    """Mesh-Conv (Eqs. 17-18): conv3x3(eta * X) + b. X: [B, Cin, H, W]."""
    eta = eta_map(p, name, delta, use_eta)
    return F.conv2d(X * eta[None], p[f"{name}.W"], p[f"{name}.b"], padding=1)


def conv1x1(p, name, X):
    W = p[f"{name}.W"]
    return F.conv2d(X, W[:, :, None, None], p[f"{name}.b"])


def trunk(p, cfg: NetConfig, t):
    h = t
    for k in range(cfg.trunk_hidden):
        h = torch.tanh(h @ p[f"trunk{k}.W"].T + p[f"trunk{k}.b"])
    return h @ p["trunk_out.W"].T + p["trunk_out.b"]  # [HW, P]


def scale_input(r):
    """r * sqrt(N) / ||r|| per sample (0 for a zero residual). r: [B, H, W]."""
    n = r[0].numel()
    nrm = torch.sqrt((r * r).sum(dim=(1, 2), keepdim=True))
    return torch.where(nrm > 0, r * math.sqrt(n) / torch.where(nrm > 0, nrm, torch.ones_like(nrm)),
                       torch.zeros_like(r))


def branch(p, cfg: NetConfig, x, feats):
    """U-Net branch on the input channels x [B, in_channels, ny, nx]; returns B(p) [B, P, ny, nx]."""
    B = x.shape[0]
    E = []
    for l in range(cfg.levels):
        delta, widths = feats[l]
        if l > 0:
            x = F.avg_pool2d(E[-1], 2)
        if cfg.use_spacing:
            x = torch.cat([x, widths[None].expand(B, -1, -1, -1)], dim=1)
        x = F.relu(mconv(p, f"enc{l}.a", x, delta, cfg.use_eta))
        x = F.relu(mconv(p, f"enc{l}.b", x, delta, cfg.use_eta))
        E.append(x)
    d = E[-1]
    for l in range(cfg.levels - 2, -1, -1):
        delta, widths = feats[l]
        u = F.interpolate(conv1x1(p, f"up{l}", d), scale_factor=2, mode="nearest")
        parts = [u, E[l]] + ([widths[None].expand(B, -1, -1, -1)] if cfg.use_spacing else [])
        x = torch.cat(parts, dim=1)
        x = F.relu(mconv(p, f"dec{l}.c", x, delta, cfg.use_eta))
        d = F.relu(mconv(p, f"dec{l}.d", x, delta, cfg.use_eta))
    return conv1x1(p, "head", d)


def net_input(r, mask):
    """[scaled residual, mask] channels, [B, 2, ny, nx]."""
    r = torch.as_tensor(r, dtype=torch.float64)
    if r.dim() == 2:
        r = r[None]
    m = torch.zeros_like(r) if mask is None else torch.as_tensor(np.asarray(mask), dtype=torch.float64).expand_as(r)
    return torch.stack([scale_input(r), m], dim=1)


def forward(p, cfg: NetConfig, grid, r, mask=None, feats=None, tin=None):
    """y = NN(r) for residual fields r [B, ny, nx] on one grid. Returns [B, ny, nx]."""
    feats = feats if feats is not None else grid_features(grid, cfg)
    Bc = branch(p, cfg, net_input(r, mask), feats)  # [B, P, H, W]
    T = trunk(p, cfg, tin if tin is not None else trunk_input(grid))  # [HW, P]
    T = T.T.reshape(1, cfg.basis, grid.ny, grid.nx)
    return p["gamma"] * (Bc * T).sum(dim=1)


def provider(p, cfg: NetConfig, grid, mask=None):
    """Error-direction provider for the hybrid oracle: r [ny, nx] -> NN(r) [ny, nx]."""
    feats = grid_features(grid, cfg)
    tin = trunk_input(grid)

    def prov(r):
        with torch.no_grad():
            return forward(p, cfg, grid, r, mask, feats, tin)[0].numpy()

    return prov


def init_params(cfg: NetConfig, rng: np.random.Generator, phi_scale=0.5):
    """Fan-in scaled random parameters (biases small), as a dict of float64 tensors."""
    p = {}
    for name, shape in param_spec(cfg):
        if name == "gamma":
            v = np.array([1.0 / math.sqrt(cfg.basis)])
        elif name.endswith(".W"):
            fan_in = int(np.prod(shape[1:]))
            gain = math.sqrt(2.0) if (name.startswith("enc") or name.startswith("dec")) and ".phi." not in name else 1.0
            if ".phi.W2" in name:
                gain = phi_scale
            v = rng.standard_normal(shape) * gain / math.sqrt(fan_in)
        else:
            v = 0.05 * rng.standard_normal(shape)
        p[name] = torch.from_numpy(np.asarray(v, dtype=np.float64))
    return p


def bf16_round(x) -> np.ndarray:
    """Nearest bfloat16 value of each float32 value (ties to the even
    significand), returned as float32.

    A bfloat16 keeps the sign, the 8 exponent bits and the top 7 fraction bits
    of a float32, i.e. the upper 16 bits of its encoding. The value is rounded
    on the discarded lower 16 bits: above half of the upper half's unit in the
    last place it rounds away from zero, below it truncates, and at exactly
    half it goes to the neighbour whose last kept bit is 0. Carries ripple into
    the exponent as in any rounding of a binary encoding."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    bits = a.view(np.uint32)
    upper = bits >> np.uint32(16)
    lower = bits & np.uint32(0xFFFF)
    half = np.uint32(0x8000)
    up = (lower > half) | ((lower == half) & ((upper & np.uint32(1)) == 1))
    upper = upper + up.astype(np.uint32)
    return (upper << np.uint32(16)).astype(np.uint32).view(np.float32).reshape(a.shape)


def round_bf16_params(cfg: NetConfig, p):
    """Copy of p with the BF16-consumed matrices rounded to BF16 values."""
    q = {}
    for name, t in p.items():
        if name in bf16_params(cfg):
            q[name] = torch.from_numpy(bf16_round(t.numpy()).astype(np.float64))
        else:
            q[name] = t.clone()
    return q


def residual_loss(p, cfg, grids, R, masks=None, apply=None):
    """Eq. 19 averaged over the batch: mean over samples and cells of (R - A NN(R))^2.

    grids: list of grids (one per sample, same size); R: [B, ny, nx];
    apply(grid, y) -> A y (FP64, differentiable through torch)."""
    total = 0.0
    for s, g in enumerate(grids):
        y = forward(p, cfg, g, R[s:s + 1], None if masks is None else masks[s])[0]
        res = torch.as_tensor(R[s], dtype=torch.float64) - apply(g, y)
        total = total + (res * res).mean()
    return total / len(grids)


def loss_and_grad(p, cfg, grids, R, masks=None, apply=None):
    """Eq. 19 loss and its gradient (autograd) at the parameters p."""
    q = {k: v.detach().clone().requires_grad_(True) for k, v in p.items()}
    loss = residual_loss(q, cfg, grids, R, masks=masks, apply=apply)
    loss.backward()
    return float(loss.detach()), {k: (v.grad.detach().clone() if v.grad is not None else torch.zeros_like(v))
                         for k, v in q.items()}


def sam_gradient(p, cfg, grids, R, rho, masks=None, apply=None, bf16=True):
    """Gradient of a sharpness-aware minimisation step (Foret et al., ICLR
    2021), which Sec. 2.4 combines with Adam: with g the gradient of the loss
    at w, the optimiser is handed the gradient at w + rho g / |g|_2, the norm
    taken over all parameters together; the update itself is applied to w.
    With bf16, the perturbed matrices the network consumes in BF16 are
    rounded as the unperturbed ones are."""
    _, g = loss_and_grad(p, cfg, grids, R, masks, apply)
    norm = math.sqrt(sum(float((t * t).sum()) for t in g.values()))
    scale = rho / norm if norm > 0 else 0.0
    w = {k: p[k].detach() + scale * g[k] for k in p}
    if bf16:
        w = round_bf16_params(cfg, w)
    return loss_and_grad(w, cfg, grids, R, masks, apply)


def supervised_loss_of(y, e):
    """Scale- and shift-invariant misfit of an output y against a target e
    (both [ny, nx]): 1 - (y0 . e0)^2 / (|y0|^2 |e0|^2) with y0, e0 the fields
    minus their means. The line search of Eqs. 12-13 is blind to the output's
    scale and to constants (A 1 = 0), so only the direction matters."""
    y0 = y - y.mean()
    e0 = e - e.mean()
    return 1.0 - (y0 * e0).sum() ** 2 / ((y0 * y0).sum() * (e0 * e0).sum())


def anorm_loss_of(y, R, e, Ay):
    """One minus the share of the A-norm error that one exact line search
    along y removes (the DLSM step of Eqs. 12-13 with residual R and error
    e = A^+ R): 1 - (R . y)^2 / ((y . A y)(R . e)). Ay is A y. Invariant to
    the scale of y and to constants in it (A 1 = 0 and R . 1 = 0). This loss
    is an option beside Eq. 19: it weights the misfit by A once, where the
    residual loss weights it by A^2."""
    return 1.0 - (R * y).sum() ** 2 / ((y * Ay).sum() * (R * e).sum())


def anorm_loss(p, cfg, grids, R, targets, masks=None, apply=None):
    """Batch mean of anorm_loss_of(NN(R_s), R_s, e_s, A NN(R_s)) with the FP64
    target e_s (the solution of A e_s = R_s); apply(grid, y) -> A y."""
    total = 0.0
    for s, g in enumerate(grids):
        y = forward(p, cfg, g, R[s:s + 1], None if masks is None else masks[s])[0]
        Rs = torch.as_tensor(R[s], dtype=torch.float64)
        total = total + anorm_loss_of(y, Rs, torch.as_tensor(targets[s], dtype=torch.float64), apply(g, y))
    return total / len(grids)


def supervised_loss(p, cfg, grids, R, targets, masks=None):
    """Batch mean of supervised_loss_of(NN(R_s), e_s) (the FP64 target e_s,
    typically the solution of A e_s = R_s)."""
    total = 0.0
    for s, g in enumerate(grids):
        y = forward(p, cfg, g, R[s:s + 1], None if masks is None else masks[s])[0]
        total = total + supervised_loss_of(y, torch.as_tensor(targets[s], dtype=torch.float64))
    return total / len(grids)
