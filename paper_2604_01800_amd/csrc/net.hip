// DeepONet host runtime: parameter layout, initialisation, persistence, the
// per-grid network constants and the forward pass (Sec. 2.4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "api_internal.hpp"
#include "net_internal.hpp"
#include "net_kernels.hpp"

namespace ppe {

static int pad8(int c) { return (c + 7) / 8 * 8; }

#define HIPCHK(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return set_error(PPE_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// Flat parameter layout, in the order: encoder levels (layers a, b), decoder
// levels L-2..0 (1x1 up-conv, layers c, d), head, trunk layers, gamma.
static void build_layout(ppe_net* n) {
  const ppe_net_config& c = n->cfg;
  const int L = c.levels, H = c.phi_hidden, sp = 2 * c.use_spacing;
  auto ch = [&](int l) { return c.base_channels << l; };
  int64_t o = 0, op = 0;
  auto mconv = [&](int level, int cin, int cout) {
    MConvL m;
    m.level = level;
    m.cin = cin;
    m.cout = cout;
    m.cin8 = pad8(cin);
    m.oW = o;
    o += (int64_t)cout * cin * 9;
    m.ob = o;
    o += cout;
    m.oW1 = o;
    o += (int64_t)H * 4;
    m.ob1 = o;
    o += H;
    m.phik = c.use_eta == 2 ? 1 : cin;
    m.oW2 = o;
    o += (int64_t)m.phik * H;
    m.ob2 = o;
    o += m.phik;
    m.kp = conv_packed_k(9, m.cin8);
    m.opack = op;
    op += (int64_t)cout * m.kp;
    return m;
  };
  n->enc_a.clear();
  n->enc_b.clear();
  n->dec_c.assign(L, MConvL{});
  n->dec_d.assign(L, MConvL{});
  n->up.assign(L, UpL{});
  for (int l = 0; l < L; ++l) {
    n->enc_a.push_back(mconv(l, (l == 0 ? 2 : ch(l - 1)) + sp, ch(l)));
    n->enc_b.push_back(mconv(l, ch(l), ch(l)));
  }
  for (int l = L - 2; l >= 0; --l) {
    UpL u;
    u.level = l;
    u.cin = ch(l + 1);
    u.cout = ch(l);
    u.oW = o;
    o += (int64_t)u.cout * u.cin;
    u.ob = o;
    o += u.cout;
    u.kp = conv_packed_k(1, u.cin);
    u.opack = op;
    op += (int64_t)u.cout * u.kp;
    n->up[l] = u;
    n->dec_c[l] = mconv(l, 2 * ch(l) + sp, ch(l));
    n->dec_d[l] = mconv(l, ch(l), ch(l));
  }
  n->o_headW = o;
  o += (int64_t)c.basis * ch(0);
  n->o_headb = o;
  o += c.basis;
  int nin = 2;
  n->o_tW.clear();
  n->o_tb.clear();
  for (int k = 0; k <= c.trunk_hidden; ++k) {
    const int nout = k == c.trunk_hidden ? c.basis : c.trunk_width;
    n->o_tW.push_back(o);
    o += (int64_t)nout * nin;
    n->o_tb.push_back(o);
    o += nout;
    nin = nout;
  }
  n->o_gamma = o;
  o += 1;
  n->np = o;
  n->npack = op;
}

// splitmix64 + Box-Muller: the library's own seeded initialisation.
static uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
static double unit(uint64_t& s) { return ((splitmix(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
static double gauss(uint64_t& s) {
  const double u = unit(s), v = unit(s);
  return std::sqrt(-2.0 * std::log(u)) * std::cos(6.283185307179586 * v);
}

static void init_params(ppe_net* n, uint64_t seed, std::vector<float>& w) {
  w.assign(n->np, 0.f);
  uint64_t s = seed ^ 0x5bd1e995u;
  auto fill = [&](int64_t o, int64_t cnt, double sd) {
    for (int64_t k = 0; k < cnt; ++k) w[o + k] = (float)(sd * gauss(s));
  };
  const int H = n->cfg.phi_hidden;
  auto mconv = [&](const MConvL& m) {
    fill(m.oW, (int64_t)m.cout * m.cin * 9, std::sqrt(2.0 / (9.0 * m.cin)));
    fill(m.oW1, (int64_t)H * 4, 0.5);
    fill(m.oW2, (int64_t)m.phik * H, 0.1 / std::sqrt((double)H));
  };
  for (auto& m : n->enc_a) mconv(m);
  for (auto& m : n->enc_b) mconv(m);
  for (int l = 0; l < n->cfg.levels - 1; ++l) {
    const UpL& u = n->up[l];
    fill(u.oW, (int64_t)u.cout * u.cin, std::sqrt(1.0 / u.cin));
    mconv(n->dec_c[l]);
    mconv(n->dec_d[l]);
  }
  const int c0 = n->cfg.base_channels;
  fill(n->o_headW, (int64_t)n->cfg.basis * c0, std::sqrt(1.0 / c0));
  int nin = 2;
  for (int k = 0; k <= n->cfg.trunk_hidden; ++k) {
    const int nout = k == n->cfg.trunk_hidden ? n->cfg.basis : n->cfg.trunk_width;
    fill(n->o_tW[k], (int64_t)nout * nin, std::sqrt(1.0 / nin));
    nin = nout;
  }
  w[n->o_gamma] = (float)(1.0 / std::sqrt((double)n->cfg.basis));
}

// Re-packs the BF16 MFMA weights from the FP32 masters and bumps the version
// (per-grid constants depending on the weights are rebuilt lazily).
ppe_status net_refresh(ppe_net* n, hipStream_t s) {
  auto pack = [&](const MConvL& m) {
    launch_pack_weights(n->d_w + m.oW, m.cout, m.cin, m.cin8, 9, m.kp, n->d_pack + m.opack, s);
  };
  for (auto& m : n->enc_a) pack(m);
  for (auto& m : n->enc_b) pack(m);
  for (int l = 0; l < n->cfg.levels - 1; ++l) {
    const UpL& u = n->up[l];
    launch_pack_weights(n->d_w + u.oW, u.cout, u.cin, u.cin, 1, u.kp, n->d_pack + u.opack, s);
    pack(n->dec_c[l]);
    pack(n->dec_d[l]);
  }
  HIPCHK(hipGetLastError());
  n->version++;
  return PPE_OK;
}

static ppe_status check_config(const ppe_net_config& c) {
  if (c.levels < 2 || c.levels > 6) return set_error(PPE_ERR_INVALID_ARG, "levels must be in [2, 6]");
  if (c.base_channels < 8 || c.base_channels % 8) return set_error(PPE_ERR_INVALID_ARG, "base_channels: multiple of 8");
  if ((int64_t)c.base_channels << (c.levels - 1) > 1024)
    return set_error(PPE_ERR_INVALID_ARG, "base_channels x 2^(levels-1) must not exceed 1024");
  // both are channel pitches of activation buffers read in 8-channel (16-byte) groups
  if (c.basis < 8 || c.basis > 128 || c.basis % 8 || c.trunk_width < 8 || c.trunk_width > 128 || c.trunk_width % 8)
    return set_error(PPE_ERR_INVALID_ARG, "basis and trunk_width must be multiples of 8 in [8, 128]");
  if (c.trunk_hidden < 1 || c.trunk_hidden > 8) return set_error(PPE_ERR_INVALID_ARG, "trunk_hidden in [1, 8]");
  if (c.phi_hidden < 1 || c.phi_hidden > 32) return set_error(PPE_ERR_INVALID_ARG, "phi_hidden in [1, 32]");
  if (c.use_eta < 0 || c.use_eta > 2) return set_error(PPE_ERR_INVALID_ARG, "use_eta in {0, 1, 2}");
  return PPE_OK;
}

// ---------------------------------------------------------------------------
// Per-grid network constants and activation buffers.

void net_cache_free(NetCache* c) {
  if (!c) return;
  dev_free(c->d_lv);
  dev_free(c->d_eta);
  dev_free(c->d_fold);
  dev_free(c->d_act);
  dev_free(c->d_part);
  dev_free(c->d_kpart);
  delete c;
}

// Level coordinates: centres average-pooled pairwise per level, widths merged;
// neighbour distances with nearest-neighbour padding; all divided by the
// level's mean spacing (length / pixels).
static void level_arrays(const std::vector<double>& xc, const std::vector<double>& hx, int levels,
                         std::vector<std::vector<float>>& dl, std::vector<std::vector<float>>& dr,
                         std::vector<std::vector<float>>& hn) {
  double Ltot = 0;
  for (double h : hx) Ltot += h;
  std::vector<double> c = xc, h = hx;
  dl.assign(levels, {});
  dr.assign(levels, {});
  hn.assign(levels, {});
  for (int l = 0; l < levels; ++l) {
    if (l > 0) {
      std::vector<double> c2(c.size() / 2), h2(h.size() / 2);
      for (size_t i = 0; i < c2.size(); ++i) {
        c2[i] = 0.5 * (c[2 * i] + c[2 * i + 1]);
        h2[i] = h[2 * i] + h[2 * i + 1];
      }
      c.swap(c2);
      h.swap(h2);
    }
    const int n = (int)c.size();
    const double sc = n / Ltot;
    dl[l].resize(n);
    dr[l].resize(n);
    hn[l].resize(n);
    for (int i = 0; i < n; ++i) {
      const double left = i > 0 ? c[i] - c[i - 1] : c[1] - c[0];
      const double right = i < n - 1 ? c[i + 1] - c[i] : c[n - 1] - c[n - 2];
      dl[l][i] = (float)(left * sc);
      dr[l][i] = (float)(right * sc);
      hn[l][i] = (float)(h[i] * sc);
    }
  }
}

// Per-grid block of 1D network inputs: for each level l the arrays
// [dxl W_l][dxr W_l][hxn W_l][dyd H_l][dyu H_l][hyn H_l] (offsets in lv_off),
// then the trunk inputs [x_hat nx][y_hat ny] (offset *tin_off).
void grid_block(const ppe_problem* p, int L, std::vector<float>& lv, int64_t* lv_off, int64_t* tin_off) {
  std::vector<std::vector<float>> xl, xr, xh, yd, yu, yh;
  level_arrays(p->xc, p->hx, L, xl, xr, xh);
  level_arrays(p->yc, p->hy, L, yd, yu, yh);
  lv.clear();
  for (int l = 0; l < L; ++l) {
    lv_off[l] = (int64_t)lv.size();
    for (auto* v : {&xl[l], &xr[l], &xh[l], &yd[l], &yu[l], &yh[l]}) lv.insert(lv.end(), v->begin(), v->end());
  }
  double Lx = 0, Ly = 0;
  for (double h : p->hx) Lx += h;
  for (double h : p->hy) Ly += h;
  const double x0 = p->xc[0] - 0.5 * p->hx[0], y0 = p->yc[0] - 0.5 * p->hy[0];
  *tin_off = (int64_t)lv.size();
  for (int i = 0; i < p->nx; ++i) lv.push_back((float)(2.0 * (p->xc[i] - x0) / Lx - 1.0));
  for (int j = 0; j < p->ny; ++j) lv.push_back((float)(2.0 * (p->yc[j] - y0) / Ly - 1.0));
}

ppe_status net_cache_ensure(ppe_problem* p, ppe_net* n, int nb, hipStream_t s) {
  const ppe_net_config& cfg = n->cfg;
  const int L = cfg.levels;
  NetCache* c = p->net_cache;
  const bool layout_ok = c && c->net_uid == n->uid && c->L == L && c->nb >= nb && c->use_eta == cfg.use_eta &&
                         c->use_spacing == cfg.use_spacing && c->c0 == cfg.base_channels;
  if (layout_ok && c->version == n->version) return PPE_OK;
  if (!layout_ok) {
    net_cache_free(c);
    p->net_cache = c = new NetCache();
    c->net_uid = n->uid;
    c->L = L;
    c->nb = nb;
    c->use_eta = cfg.use_eta;
    c->use_spacing = cfg.use_spacing;
    c->c0 = cfg.base_channels;
    for (int l = 0; l < L; ++l) {
      c->H[l] = p->ny >> l;
      c->W[l] = p->nx >> l;
    }
    std::vector<float> lv;
    grid_block(p, L, lv, c->lv_off, &c->tin_off);
    c->d_lv = (float*)dev_alloc(lv.size() * sizeof(float));
    if (!c->d_lv) return set_error(PPE_ERR_HIP, "allocation of level arrays failed");
    HIPCHK(hipMemcpy(c->d_lv, lv.data(), lv.size() * sizeof(float), hipMemcpyHostToDevice));
    // Channel pitches: the level inputs past level 0 hold only the pooled
    // features and the decoder concatenations only the upsampled and skip
    // features; the two static channels (widths) of each level live in a
    // buffer of their own (pitch 8), the convolutions' second input source.
    // So every kernel that writes features into these buffers writes whole
    // channel groups of pixel records that start on 64-byte boundaries (for
    // base channels a multiple of 32), and the readers read no padding.
    for (int l = 0; l < L; ++l) {
      c->p_in[l] = l == 0 ? n->enc_a[l].cin8 : (cfg.base_channels << (l - 1));
      if (l < L - 1) c->p_cat[l] = 2 * (cfg.base_channels << l);
    }
    // eta maps, one per Mesh-Conv layer (shared by the batch); per-channel
    // maps have the layer's cin8 channels per pixel
    int64_t eo = 0;
    auto eta_slot = [&](const MConvL& m) {
      const int64_t o = eo;
      eo += (int64_t)c->H[m.level] * c->W[m.level] * (cfg.use_eta == 2 ? 1 : m.cin8);
      eo = (eo + 63) / 64 * 64;
      return o;
    };
    for (int l = 0; l < L; ++l) {
      c->eta_a[l] = eta_slot(n->enc_a[l]);
      c->eta_b[l] = eta_slot(n->enc_b[l]);
      if (l < L - 1) {
        c->eta_c[l] = eta_slot(n->dec_c[l]);
        c->eta_d[l] = eta_slot(n->dec_d[l]);
      }
    }
    if (cfg.use_eta) {
      c->d_eta = (bf16_t*)dev_alloc(eo * sizeof(bf16_t));
      if (!c->d_eta) return set_error(PPE_ERR_HIP, "allocation of eta maps failed");
    }
    c->fold_pitch = (cfg.base_channels + 1 + 3) & ~3;  // C0 weights and the constant term, padded to 4 floats
    c->d_fold = (float*)dev_alloc((size_t)p->nx * p->ny * c->fold_pitch * sizeof(float));
    if (!c->d_fold) return set_error(PPE_ERR_HIP, "allocation of the trunk basis failed");
    // activation buffers for nb samples
    int64_t ao = 0;
    auto act = [&](int l, int pitch) {
      const int64_t o = ao;
      ao += (int64_t)c->H[l] * c->W[l] * pitch * nb;
      ao = (ao + 127) / 128 * 128;
      return o;
    };
    for (int l = 0; l < L; ++l) {
      const int ch = cfg.base_channels << l;
      c->o_in[l] = act(l, c->p_in[l]);
      c->o_a[l] = act(l, ch);
      if (l < L - 1) {
        c->o_cat[l] = act(l, c->p_cat[l]);
        c->o_c[l] = act(l, ch);
        c->o_d[l] = act(l, ch);
        c->o_up[l] = act(l + 1, ch);  // the up-convolution's output, at level l + 1's resolution
      } else {
        c->o_bot = act(l, ch);
      }
      if (cfg.use_spacing) {  // one copy for the batch
        c->o_st[l] = ao;
        ao += (int64_t)c->H[l] * c->W[l] * 8;
        ao = (ao + 127) / 128 * 128;
      }
    }
    c->act_elems = ao;
    c->d_act = (bf16_t*)dev_alloc(ao * sizeof(bf16_t));
    c->d_part = (double*)dev_alloc((size_t)kRedBlocks * nb * sizeof(double));
    c->kpart_elems = conv_kpart_elems();
    c->d_kpart = (float*)dev_alloc((size_t)c->kpart_elems * sizeof(float));
    if (!c->d_act || !c->d_part || !c->d_kpart)
      return set_error(PPE_ERR_HIP, "allocation of network activations failed");
    HIPCHK(hipMemsetAsync(c->d_act, 0, ao * sizeof(bf16_t), s));
    // static channels: widths (and the mask at level 0, in the level-0
    // input; the widths of every level also in the level's static buffer)
    for (int l = 0; l < L; ++l) {
      const float* hxn = c->d_lv + c->lv_off[l] + 2 * c->W[l];
      const float* hyn = c->d_lv + c->lv_off[l] + 3 * c->W[l] + 2 * c->H[l];
      if (l == 0) {
        const int64_t bs_in = (int64_t)c->H[0] * c->W[0] * c->p_in[0];
        launch_fill_static(c->H[0], c->W[0], c->p_in[0], cfg.use_spacing ? 2 : -1, hxn, hyn, p->d_mask, 1,
                           c->d_act + c->o_in[0], bs_in, nb, s);
      }
      if (cfg.use_spacing)
        launch_fill_static(c->H[l], c->W[l], 8, 0, hxn, hyn, nullptr, -1, c->d_act + c->o_st[l], 0, 1, s);
    }
    HIPCHK(hipGetLastError());
  }
  // weight-dependent constants: eta maps and the folded trunk basis
  if (cfg.use_eta) {
    auto eta = [&](const MConvL& m, int64_t off) {
      const int l = m.level;
      const float* b = c->d_lv + c->lv_off[l];
      const int W = c->W[l], H = c->H[l];
      // one weight per pixel: the same kernel with one output channel
      const int k = m.phik, k8 = cfg.use_eta == 2 ? 1 : m.cin8;
      launch_eta(H, W, k, k8, cfg.phi_hidden, b, b + W, b + 3 * W, b + 3 * W + H, n->d_w + m.oW1, n->d_w + m.ob1,
                 n->d_w + m.oW2, n->d_w + m.ob2, c->d_eta + off, s);
    };
    for (int l = 0; l < L; ++l) {
      eta(n->enc_a[l], c->eta_a[l]);
      eta(n->enc_b[l], c->eta_b[l]);
      if (l < L - 1) {
        eta(n->dec_c[l], c->eta_c[l]);
        eta(n->dec_d[l], c->eta_d[l]);
      }
    }
  }
  TrunkDesc td{};
  td.hidden = cfg.trunk_hidden;
  td.width = cfg.trunk_width;
  td.basis = cfg.basis;
  td.c0 = cfg.base_channels;
  td.fold_pitch = c->fold_pitch;
  for (int k = 0; k <= cfg.trunk_hidden; ++k) {
    td.oW[k] = n->o_tW[k];
    td.ob[k] = n->o_tb[k];
  }
  td.oWh = n->o_headW;
  td.obh = n->o_headb;
  launch_trunk_fold(p->ny, p->nx, c->d_lv + c->tin_off, c->d_lv + c->tin_off + p->nx, n->d_w, td, c->d_fold, s);
  HIPCHK(hipGetLastError());
  c->version = n->version;
  return PPE_OK;
}

static ConvGeo geo(const NetCache* c, int l, int cin8, int cout, int y_pitch, int y_off, int nb_eta_shared,
                   int x_pitch = 0) {
  ConvGeo g{};
  g.H = c->H[l];
  g.W = c->W[l];
  g.cin8 = cin8;
  g.x_pitch = x_pitch ? x_pitch : cin8;
  g.c1 = cin8;
  g.x1_pitch = 0;
  g.x1 = nullptr;
  g.x1_bstride = 0;
  g.cout = cout;
  g.y_pitch = y_pitch;
  g.y_off = y_off;
  g.x_bstride = (int64_t)g.H * g.W * g.x_pitch;
  g.y_bstride = (int64_t)g.H * g.W * y_pitch;
  g.eta_node = c->use_eta == 2;
  g.e_bstride = nb_eta_shared ? 0 : (int64_t)g.H * g.W * (g.eta_node ? 1 : cin8);
  g.act = 1;
  return g;
}

// A convolution whose input channels past the feature buffer's pitch are
// the level's static channels (the second input source, shared by the batch).
static ConvGeo with_static(const NetCache* c, ConvGeo g, int l, const bf16_t* A) {
  if (g.x_pitch < g.cin8) {
    g.c1 = g.x_pitch;
    g.x1 = A + c->o_st[l];
    g.x1_pitch = 8;
    g.x1_bstride = 0;
  }
  return g;
}

// One launch of the forward on one grid: what the launch over nb samples of
// the grid, or a grouped launch over grids, needs.
struct FwdOp {
  enum Kind { PACK, CONV, OUT } kind = PACK;
  // PACK: channel 0 of the level-0 input from r (pitch, bstride)
  const float* r = nullptr;
  int64_t n = 0;
  double* part = nullptr;
  bf16_t* xin = nullptr;
  int pitch = 0;
  int64_t bstride = 0;
  // CONV
  int taps = 9;
  bool up = false;
  ConvGeo g{};
  const bf16_t* x = nullptr;
  const bf16_t* eta = nullptr;
  const bf16_t* wp = nullptr;
  int Kp = 0;
  const float* bias = nullptr;
  bf16_t* y = nullptr;
  float* kpart = nullptr;
  int64_t kpart_elems = 0;
  int tn = 0;  // output channels per workgroup (0: the default)
  // OUT
  int c0 = 0, fold_pitch = 0;
  const bf16_t* d0 = nullptr;
  int64_t d_bs = 0;
  const float* fold = nullptr;
  const float* gamma = nullptr;
  float* yout = nullptr;
};

// The forward's launches for the grid of cache c, in order: input scaling,
// per encoder level two Mesh-Convs (the second also writes the 2 x 2 average
// of its output, E_l, as the next level's input), per decoder level the 1x1
// up-convolution and two Mesh-Convs, then the DeepONet output.
static void forward_ops(const ppe_problem* p, const ppe_net* n, const NetCache* c, const float* r, float* y,
                        std::vector<FwdOp>& ops) {
  const ppe_net_config& cfg = n->cfg;
  const int L = cfg.levels;
  const int64_t N = (int64_t)p->nx * p->ny;
  bf16_t* A = c->d_act;
  const bf16_t* E = c->d_eta;
  auto ch = [&](int l) { return cfg.base_channels << l; };
  auto eta = [&](int64_t off) -> const bf16_t* { return cfg.use_eta ? E + off : nullptr; };
  ops.clear();
  FwdOp pk;
  pk.kind = FwdOp::PACK;
  pk.r = r;
  pk.n = N;
  pk.part = c->d_part;
  pk.xin = A + c->o_in[0];
  pk.pitch = c->p_in[0];
  pk.bstride = N * c->p_in[0];
  ops.push_back(pk);
  auto conv = [&](int taps, bool up, const ConvGeo& g, const bf16_t* x, const bf16_t* e, const bf16_t* wp, int Kp,
                  const float* bias, bf16_t* yo) {
    FwdOp o;
    o.kind = FwdOp::CONV;
    o.taps = taps;
    o.up = up;
    o.g = g;
    o.x = x;
    o.eta = e;
    o.wp = wp;
    o.Kp = Kp;
    o.bias = bias;
    o.y = yo;
    o.kpart = c->d_kpart;
    o.kpart_elems = c->kpart_elems;
    o.tn = ops.size() < sizeof(c->conv_tn) ? c->conv_tn[ops.size()] : 0;
    ops.push_back(o);
  };
  for (int l = 0; l < L; ++l) {
    const int64_t hw = (int64_t)c->H[l] * c->W[l];
    const MConvL& ma = n->enc_a[l];
    const MConvL& mb = n->enc_b[l];
    conv(9, false, with_static(c, geo(c, l, ma.cin8, ma.cout, ch(l), 0, 1, c->p_in[l]), l, A), A + c->o_in[l],
         eta(c->eta_a[l]), n->d_pack + ma.opack, ma.kp, n->d_w + ma.ob, A + c->o_a[l]);
    if (l < L - 1) {
      // E_l into the decoder concat buffer of level l at channel C_l, and pooled into level l + 1
      ConvGeo gb = geo(c, l, mb.cin8, mb.cout, c->p_cat[l], ch(l), 1);
      gb.pool_y = A + c->o_in[l + 1];
      gb.pool_pitch = c->p_in[l + 1];
      gb.pool_bstride = (int64_t)c->H[l + 1] * c->W[l + 1] * c->p_in[l + 1];
      conv(9, false, gb, A + c->o_a[l], eta(c->eta_b[l]), n->d_pack + mb.opack, mb.kp, n->d_w + mb.ob,
           A + c->o_cat[l]);
    }
    else
      conv(9, false, geo(c, l, mb.cin8, mb.cout, ch(l), 0, 1), A + c->o_a[l], eta(c->eta_b[l]), n->d_pack + mb.opack,
           mb.kp, n->d_w + mb.ob, A + c->o_bot);
  }
  for (int l = L - 2; l >= 0; --l) {
    const UpL& u = n->up[l];
    const bf16_t* src = (l == L - 2) ? A + c->o_bot : A + c->o_d[l + 1];
    // the 1x1 up-convolution at the coarse level; the next convolution reads
    // its output through the nearest upsampling as its first C_l channels
    ConvGeo gu = geo(c, l + 1, u.cin, u.cout, ch(l), 0, 1);
    gu.act = 0;
    conv(1, false, gu, src, nullptr, n->d_pack + u.opack, u.kp, n->d_w + u.ob, A + c->o_up[l]);
    const MConvL& mc = n->dec_c[l];
    const MConvL& md = n->dec_d[l];
    ConvGeo gc = with_static(c, geo(c, l, mc.cin8, mc.cout, ch(l), 0, 1, c->p_cat[l]), l, A);
    gc.xu = A + c->o_up[l];
    gc.cu = ch(l);
    gc.xu_pitch = ch(l);
    gc.xu_bstride = (int64_t)c->H[l + 1] * c->W[l + 1] * ch(l);
    conv(9, false, gc, A + c->o_cat[l], eta(c->eta_c[l]), n->d_pack + mc.opack, mc.kp, n->d_w + mc.ob, A + c->o_c[l]);
    conv(9, false, geo(c, l, md.cin8, md.cout, ch(l), 0, 1), A + c->o_c[l], eta(c->eta_d[l]), n->d_pack + md.opack,
         md.kp, n->d_w + md.ob, A + c->o_d[l]);
  }
  FwdOp o;
  o.kind = FwdOp::OUT;
  o.n = N;
  o.c0 = cfg.base_channels;
  o.d0 = A + c->o_d[0];
  o.d_bs = N * cfg.base_channels;
  o.fold = c->d_fold;
  o.fold_pitch = c->fold_pitch;
  o.gamma = n->d_w + n->o_gamma;
  o.yout = y;
  ops.push_back(o);
}

// One launch of the forward over nb samples.
static void launch_op(const FwdOp& o, int nb, hipStream_t s) {
  switch (o.kind) {
    case FwdOp::PACK: launch_input_pack(o.r, o.n, nb, o.part, o.xin, o.pitch, o.bstride, s); break;
    case FwdOp::CONV:
      launch_conv(o.taps, o.up, o.g, nb, o.x, o.eta, o.wp, o.Kp, o.bias, o.y, s, o.kpart, o.kpart_elems, o.tn);
      break;
    case FwdOp::OUT: launch_deeponet_out(o.n, o.c0, o.d0, o.d_bs, o.fold, o.fold_pitch, o.gamma, o.yout, nb, s); break;
  }
}

// y = NN(r) for nb residual fields of one grid (device FP32 in and out).
ppe_status net_forward(ppe_problem* p, ppe_net* n, int nb, const float* r, float* y, hipStream_t s) {
  ppe_status st = net_cache_ensure(p, n, nb, s);
  if (st != PPE_OK) return st;
  std::vector<FwdOp> ops;
  forward_ops(p, n, p->net_cache, r, y, ops);
  // the last decoder convolution computes the DeepONet output in its
  // epilogue where the layer allows it (same values as the two launches)
  const size_t no = ops.size();
  const bool fuse = no >= 2 && ops[no - 1].kind == FwdOp::OUT && ops[no - 2].kind == FwdOp::CONV &&
                    ops[no - 2].taps == 9 && !ops[no - 2].up && ops[no - 2].y == ops[no - 1].d0;
  for (size_t k = 0; k < (fuse ? no - 2 : no); ++k) launch_op(ops[k], nb, s);
  if (fuse) {
    const FwdOp& cv = ops[no - 2];
    const FwdOp& ot = ops[no - 1];
    const OutFold of{ot.fold, ot.gamma, ot.yout, ot.fold_pitch, ot.c0};
    if (!launch_conv_out(cv.g, nb, cv.x, cv.eta, cv.wp, cv.Kp, cv.bias, cv.y, s, cv.kpart, cv.kpart_elems, cv.tn,
                         of)) {
      launch_op(cv, nb, s);
      launch_op(ot, nb, s);
    }
  }
  HIPCHK(hipGetLastError());
  return PPE_OK;
}

// Tile-width tuning of the forward's convolutions on one grid (see
// ppe_tune_net): each launch with a choice timed alone with either width.
static ppe_status tune_net_impl(ppe_problem* p, ppe_net* n, int nb, int reps, ppe_net_tune_result* out,
                                hipStream_t s) {
  ppe_status st = net_cache_ensure(p, n, nb, s);
  if (st != PPE_OK) return st;
  NetCache* c = p->net_cache;
  const int64_t N = (int64_t)p->nx * p->ny;
  float* r = (float*)dev_alloc((size_t)nb * N * sizeof(float) * 2);
  if (!r) return set_error(PPE_ERR_HIP, "allocation of the tuning fields failed");
  float* y = r + (size_t)nb * N;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto done = [&](ppe_status res) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    dev_free(r);
    return res;
  };
  if (hipMemsetAsync(r, 0, (size_t)nb * N * sizeof(float), s) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess)
    return done(set_error(PPE_ERR_HIP, "tuning set-up failed"));
  std::vector<FwdOp> ops;
  for (int8_t& t : c->conv_tn) t = 0;
  forward_ops(p, n, c, r, y, ops);
  if (ops.size() > sizeof(c->conv_tn)) return done(set_error(PPE_ERR_UNSUPPORTED, "too many launches to tune"));
  for (const FwdOp& o : ops) launch_op(o, nb, s);  // every buffer holds its layer's output
  if (out) {
    std::memset(out, 0, sizeof(*out));
    out->n = (int32_t)ops.size();
  }
  for (size_t k = 0; k < ops.size(); ++k) {
    FwdOp o = ops[k];
    if (o.kind != FwdOp::CONV || !conv_has_tile_choice(o.taps, o.up, o.eta != nullptr, o.g, o.Kp)) continue;
    float us[2] = {0.f, 0.f};
    for (int w = 0; w < 2; ++w) {
      o.tn = w ? 64 : 32;
      launch_op(o, nb, s);  // warm-up
      if (hipEventRecord(e0, s) != hipSuccess) return done(set_error(PPE_ERR_HIP, "hipEventRecord failed"));
      for (int i = 0; i < reps; ++i) launch_op(o, nb, s);
      float ms = 0.f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        return done(set_error(PPE_ERR_HIP, "timing of launch %zu failed", k));
      us[w] = ms * 1e3f / (float)reps;
    }
    // the default width unless the other is more than 3 % faster
    const int def = conv_default_tile(o.g, nb);
    const float ud = def == 64 ? us[1] : us[0], uo = def == 64 ? us[0] : us[1];
    const int choice = uo < 0.97f * ud ? 96 - def : def;
    c->conv_tn[k] = (int8_t)choice;
    if (out) {
      out->tile[k] = choice;
      out->us32[k] = us[0];
      out->us64[k] = us[1];
    }
  }
  if (hipGetLastError() != hipSuccess) return done(set_error(PPE_ERR_HIP, "tuning launches failed"));
  return done(PPE_OK);
}

// ---------------------------------------------------------------------------
// Grouped forward over several grids (one residual field each): the same
// launches as net_forward on each grid, each layer as one launch over all
// grids. The member tables of every layer live in one device block.

void net_group_free(NetGroup& G) {
  if (G.d_tab) (void)hipFree(G.d_tab);
  G = NetGroup{};
}

// The tables of one part (members idx of the group) appended to blob.
static ppe_status group_part(const std::vector<std::vector<FwdOp>>& ops, const std::vector<int>& idx,
                             const int32_t* const* skip, std::vector<char>& blob, GroupPart& P) {
  const int n = (int)idx.size();
  const size_t nops = ops[idx[0]].size();
  auto append = [&](const void* src, size_t bytes) {
    const size_t o = (blob.size() + 255) / 256 * 256;
    blob.resize(o + bytes);
    std::memcpy(blob.data() + o, src, bytes);
    return (int64_t)o;
  };
  auto sk = [&](int i) { return skip ? skip[idx[i]] : nullptr; };
  P.n = n;
  P.ops.resize(nops);
  for (size_t k = 0; k < nops; ++k) {
    const FwdOp& o0 = ops[idx[0]][k];
    GroupOp& q = P.ops[k];
    q.kind = o0.kind;
    switch (o0.kind) {
      case FwdOp::PACK: {
        std::vector<PackMember> m(n);
        for (int i = 0; i < n; ++i) {
          const FwdOp& o = ops[idx[i]][k];
          m[i] = PackMember{o.r, o.n, o.part, o.xin, sk(i)};
        }
        q.a = o0.pitch;
        q.off = append(m.data(), m.size() * sizeof(PackMember));
        break;
      }
      case FwdOp::CONV: {
        std::vector<ConvMember> m(n);
        for (int i = 0; i < n; ++i) {
          const FwdOp& o = ops[idx[i]][k];
          m[i] = ConvMember{};
          m[i].g = o.g;
          m[i].x = o.x;
          m[i].eta = o.eta;
          m[i].y = o.y;
          m[i].kpart = o.kpart;
          m[i].tn = o.tn;
          m[i].skip = sk(i);
        }
        if (!plan_conv_group(o0.taps, o0.up, o0.Kp, m, o0.kpart_elems, q.conv))
          return set_error(PPE_ERR_UNSUPPORTED, "layer %zu has no grouped form", k);
        q.wp = o0.wp;
        q.Kp = o0.Kp;
        q.bias = o0.bias;
        q.off = append(m.data(), m.size() * sizeof(ConvMember));
        break;
      }
      case FwdOp::OUT: {
        std::vector<OutMember> m(n);
        for (int i = 0; i < n; ++i) {
          const FwdOp& o = ops[idx[i]][k];
          m[i] = OutMember{o.n, o.d0, o.fold, o.yout, sk(i)};
          q.maxn = std::max<int64_t>(q.maxn, o.n);
        }
        q.a = o0.c0;
        q.b = o0.fold_pitch;
        q.gamma = o0.gamma;
        q.off = append(m.data(), m.size() * sizeof(OutMember));
        break;
      }
    }
  }
  return PPE_OK;
}

ppe_status net_group_build(int n, ppe_problem* const* probs, ppe_net* net, const float* const* r, float* const* y,
                           const int32_t* const* skip, hipStream_t s, NetGroup& G) {
  net_group_free(G);
  if (n < 1) return set_error(PPE_ERR_INVALID_ARG, "empty group");
  std::vector<std::vector<FwdOp>> ops(n);
  for (int i = 0; i < n; ++i) {
    ppe_status st = net_cache_ensure(probs[i], net, 1, s);
    if (st != PPE_OK) return st;
    forward_ops(probs[i], net, probs[i]->net_cache, r[i], y[i], ops[i]);
    if (ops[i].size() != ops[0].size()) return set_error(PPE_ERR_UNSUPPORTED, "group members with different layers");
  }
  // parts: first fit over the grids by decreasing size
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  auto cells = [&](int i) { return (int64_t)probs[i]->nx * probs[i]->ny; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cells(a) > cells(b); });
  std::vector<std::vector<int>> bins;
  std::vector<int64_t> fill;
  for (int i : order) {
    size_t b = 0;
    while (b < bins.size() && fill[b] + cells(i) > kGroupCells) ++b;
    if (b == bins.size()) {
      bins.emplace_back();
      fill.push_back(0);
    }
    bins[b].push_back(i);
    fill[b] += cells(i);
  }
  std::vector<char> blob;
  G.n = n;
  G.parts.resize(bins.size());
  for (size_t b = 0; b < bins.size(); ++b) {
    ppe_status st = group_part(ops, bins[b], skip, blob, G.parts[b]);
    if (st != PPE_OK) return st;
  }
  G.d_tab = (char*)dev_alloc(blob.size());
  if (!G.d_tab) return set_error(PPE_ERR_HIP, "allocation of the group tables failed");
  G.h_tab = std::move(blob);
  HIPCHK(hipMemcpyAsync(G.d_tab, G.h_tab.data(), G.h_tab.size(), hipMemcpyHostToDevice, s));
  return PPE_OK;
}

ppe_status net_group_forward(const NetGroup& G, hipStream_t s) {
  for (const GroupPart& P : G.parts)
    for (const GroupOp& q : P.ops) {
      const void* t = G.d_tab + q.off;
      switch (q.kind) {
        case FwdOp::PACK: launch_input_pack_group((const PackMember*)t, P.n, q.a, s); break;
        case FwdOp::CONV: launch_conv_group(q.conv, (const ConvMember*)t, q.wp, q.Kp, q.bias, s); break;
        case FwdOp::OUT: launch_deeponet_out_group((const OutMember*)t, P.n, q.maxn, q.a, q.b, q.gamma, s); break;
      }
    }
  HIPCHK(hipGetLastError());
  return PPE_OK;
}

ppe_status check_net_grid(const ppe_problem* p, const ppe_net* n) {
  const int L = n->cfg.levels, m = 1 << (L - 1);
  if (p->nx % m || p->ny % m || p->nx / m < 2 || p->ny / m < 2)
    return set_error(PPE_ERR_SHAPE, "grid %d x %d: nx, ny must be divisible by %d with at least 2 cells per "
                                    "axis at the coarsest level", p->nx, p->ny, m);
  return PPE_OK;
}

}  // namespace ppe

using namespace ppe;

extern "C" {

void ppe_net_config_default(ppe_net_config* c) {
  if (!c) return;
  c->levels = 4;
  c->base_channels = 32;
  c->basis = 128;
  c->trunk_width = 128;
  c->trunk_hidden = 4;
  c->phi_hidden = 16;
  c->use_eta = 2;
  c->use_spacing = 1;
}

ppe_status ppe_net_create(const ppe_net_config* cfg, uint64_t seed, ppe_net** out) {
  if (!out) return set_error(PPE_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  ppe_net_config c;
  ppe_net_config_default(&c);
  if (cfg) c = *cfg;
  ppe_status st = check_config(c);
  if (st != PPE_OK) return st;
  static std::atomic<uint64_t> next_uid{1};
  ppe_net* n = new ppe_net();
  n->uid = next_uid++;
  n->cfg = c;
  build_layout(n);
  n->d_w = (float*)dev_alloc(n->np * sizeof(float));
  n->d_g = (float*)dev_alloc(n->np * sizeof(float));
  n->d_m = (float*)dev_alloc(n->np * sizeof(float));
  n->d_v = (float*)dev_alloc(n->np * sizeof(float));
  n->d_pack = (bf16_t*)dev_alloc(n->npack * sizeof(bf16_t));
  if (!n->d_w || !n->d_g || !n->d_m || !n->d_v || !n->d_pack) {
    ppe_net_destroy(n);
    return set_error(PPE_ERR_HIP, "device allocation of the network failed");
  }
  std::vector<float> w;
  init_params(n, seed, w);
  st = ppe_net_set_params(n, w.data(), n->np);
  if (st != PPE_OK) {
    ppe_net_destroy(n);
    return st;
  }
  *out = n;
  return PPE_OK;
}

void ppe_net_destroy(ppe_net* n) {
  if (!n) return;
  dev_free(n->d_w);
  dev_free(n->d_g);
  dev_free(n->d_m);
  dev_free(n->d_v);
  dev_free(n->d_pack);
  net_train_free(n);
  delete n;
}

int64_t ppe_net_num_params(const ppe_net* n) { return n ? n->np : -1; }

ppe_status ppe_net_set_params(ppe_net* n, const float* host, int64_t count) {
  if (!n || !host) return set_error(PPE_ERR_INVALID_ARG, "net or params NULL");
  if (count != n->np) return set_error(PPE_ERR_INVALID_ARG, "expected %lld parameters, got %lld", (long long)n->np,
                                       (long long)count);
  HIPCHK(hipMemcpy(n->d_w, host, n->np * sizeof(float), hipMemcpyHostToDevice));
  HIPCHK(hipMemset(n->d_m, 0, n->np * sizeof(float)));
  HIPCHK(hipMemset(n->d_v, 0, n->np * sizeof(float)));
  HIPCHK(hipMemset(n->d_g, 0, n->np * sizeof(float)));
  n->step = 0;
  ppe_status st = net_refresh(n, 0);
  if (st != PPE_OK) return st;
  HIPCHK(hipDeviceSynchronize());
  return PPE_OK;
}

ppe_status ppe_net_get_params(const ppe_net* n, float* host, int64_t count) {
  if (!n || !host) return set_error(PPE_ERR_INVALID_ARG, "net or params NULL");
  if (count != n->np) return set_error(PPE_ERR_INVALID_ARG, "expected %lld parameters", (long long)n->np);
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(host, n->d_w, n->np * sizeof(float), hipMemcpyDeviceToHost));
  return PPE_OK;
}

// File: "PPENET01", config, step, parameter count, FP32 params, Adam m, Adam v.
ppe_status ppe_net_save(const ppe_net* n, const char* path) {
  if (!n || !path) return set_error(PPE_ERR_INVALID_ARG, "net or path NULL");
  std::vector<float> w(n->np), m(n->np), v(n->np);
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(w.data(), n->d_w, n->np * 4, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(m.data(), n->d_m, n->np * 4, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(v.data(), n->d_v, n->np * 4, hipMemcpyDeviceToHost));
  FILE* f = fopen(path, "wb");
  if (!f) return set_error(PPE_ERR_INVALID_ARG, "cannot open %s for writing", path);
  bool ok = fwrite("PPENET01", 1, 8, f) == 8 && fwrite(&n->cfg, sizeof n->cfg, 1, f) == 1 &&
            fwrite(&n->step, sizeof n->step, 1, f) == 1 && fwrite(&n->np, sizeof n->np, 1, f) == 1 &&
            fwrite(w.data(), 4, n->np, f) == (size_t)n->np && fwrite(m.data(), 4, n->np, f) == (size_t)n->np &&
            fwrite(v.data(), 4, n->np, f) == (size_t)n->np;
  ok = (fclose(f) == 0) && ok;
  return ok ? PPE_OK : set_error(PPE_ERR_INVALID_ARG, "write to %s failed", path);
}

ppe_status ppe_net_load(ppe_net* n, const char* path) {
  if (!n || !path) return set_error(PPE_ERR_INVALID_ARG, "net or path NULL");
  FILE* f = fopen(path, "rb");
  if (!f) return set_error(PPE_ERR_INVALID_ARG, "cannot open %s", path);
  char magic[8];
  ppe_net_config c;
  int64_t step = 0, np = 0;
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "PPENET01", 8) == 0 && fread(&c, sizeof c, 1, f) == 1 &&
            fread(&step, sizeof step, 1, f) == 1 && fread(&np, sizeof np, 1, f) == 1;
  if (!ok || memcmp(&c, &n->cfg, sizeof c) != 0 || np != n->np) {
    fclose(f);
    return set_error(PPE_ERR_INVALID_ARG, "%s does not hold a network of this configuration", path);
  }
  std::vector<float> w(np), m(np), v(np);
  ok = fread(w.data(), 4, np, f) == (size_t)np && fread(m.data(), 4, np, f) == (size_t)np &&
       fread(v.data(), 4, np, f) == (size_t)np;
  fclose(f);
  if (!ok) return set_error(PPE_ERR_INVALID_ARG, "%s is truncated", path);
  ppe_status st = ppe_net_set_params(n, w.data(), np);
  if (st != PPE_OK) return st;
  HIPCHK(hipMemcpy(n->d_m, m.data(), np * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(n->d_v, v.data(), np * 4, hipMemcpyHostToDevice));
  n->step = step;
  return PPE_OK;
}

ppe_status ppe_net_forward_batch(ppe_net* n, int32_t count, ppe_problem* const* problems, const float* const* r,
                                 float* const* y, hipStream_t s) {
  if (!n || count < 0 || (count > 0 && (!problems || !r || !y)))
    return set_error(PPE_ERR_INVALID_ARG, "NULL argument or negative count");
  for (int i = 0; i < count; ++i) {
    if (!problems[i] || !r[i] || !y[i]) return set_error(PPE_ERR_INVALID_ARG, "NULL entry %d", i);
    for (int j = 0; j < i; ++j)
      if (problems[j] == problems[i]) return set_error(PPE_ERR_INVALID_ARG, "problem %d repeated", i);
    const ppe_status st = check_net_grid(problems[i], n);
    if (st != PPE_OK) return st;
  }
  if (count == 0) return PPE_OK;
  NetGroup G;
  ppe_status st = net_group_build(count, problems, n, r, y, nullptr, s, G);
  if (st == PPE_OK) st = net_group_forward(G, s);
  const hipError_t e = hipStreamSynchronize(s);  // the tables are in use until the launches end
  net_group_free(G);
  if (st != PPE_OK) return st;
  if (e != hipSuccess) return set_error(PPE_ERR_HIP, "hipStreamSynchronize failed: %s", hipGetErrorString(e));
  return PPE_OK;
}

ppe_status ppe_tune_net(ppe_net* n, ppe_problem* p, int32_t nb, int32_t reps, ppe_net_tune_result* out,
                        hipStream_t s) {
  if (!n || !p) return set_error(PPE_ERR_INVALID_ARG, "net or problem NULL");
  if (nb < 1 || nb > 4096 || reps < 1 || reps > 1000)
    return set_error(PPE_ERR_INVALID_ARG, "nb in [1, 4096] and reps in [1, 1000]");
  ppe_status st = check_net_grid(p, n);
  if (st != PPE_OK) return st;
  return tune_net_impl(p, n, nb, reps, out, s);
}

ppe_status ppe_net_forward(ppe_net* n, ppe_problem* p, int32_t nb, const float* r, float* y, hipStream_t s) {
  if (!n || !p) return set_error(PPE_ERR_INVALID_ARG, "net or problem NULL");
  if (nb < 0 || (nb > 0 && (!r || !y))) return set_error(PPE_ERR_INVALID_ARG, "bad batch or buffers");
  ppe_status st = check_net_grid(p, n);
  if (st != PPE_OK) return st;
  if (nb == 0) return PPE_OK;
  return net_forward(p, n, nb, r, y, s);
}

}  // extern "C"
