// One training step of the DeepONet on nb fabricated systems (Sec. 2.4):
// BF16 forward with saved activations (each sample on its own grid), the
// residual loss of Eq. 19, Loss = mean over samples and cells of (R - A NN(R))^2,
// the hand-written backward pass, and Adam (Kingma & Ba 2015) on FP32 masters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "api_internal.hpp"
#include "kernels.hpp"
#include "net_internal.hpp"
#include "net_kernels.hpp"
#include "train_kernels.hpp"

namespace ppe {

#define HIPCHK(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return set_error(PPE_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// Training workspace for one (batch, grid size).
struct TrainState {
  int nb = 0, nx = 0, ny = 0, L = 0;
  int H[kMaxLevels] = {}, W[kMaxLevels] = {};
  int64_t lv_stride = 0, lv_off[kMaxLevels] = {}, tin_off = 0;
  float* d_lv = nullptr;           // [nb][lv_stride]
  Coef* d_coefs = nullptr;         // [nb]
  const uint8_t** d_masks = nullptr;  // [nb] device pointers (or NULL entries)
  // BF16 activations, gradients and per-sample eta maps
  bf16_t* act = nullptr;
  bf16_t* grad = nullptr;
  bf16_t* eta = nullptr;
  int p_in[kMaxLevels] = {}, p_cat[kMaxLevels] = {};
  int64_t o_in[kMaxLevels] = {}, o_a[kMaxLevels] = {}, o_cat[kMaxLevels] = {}, o_c[kMaxLevels] = {},
          o_d[kMaxLevels] = {}, o_bot = 0, o_B = 0, o_T = 0, o_t0 = 0, o_h[9] = {};
  int64_t g_in[kMaxLevels] = {}, g_a[kMaxLevels] = {}, g_cat[kMaxLevels] = {}, g_c[kMaxLevels] = {},
          g_d[kMaxLevels] = {}, g_E[kMaxLevels] = {}, g_Uc[kMaxLevels] = {}, g_bot = 0, g_B = 0, g_T = 0,
          g_h[9] = {};
  int64_t e_a[kMaxLevels] = {}, e_b[kMaxLevels] = {}, e_c[kMaxLevels] = {}, e_d[kMaxLevels] = {};
  // packed BF16 weights for this step: transposed (input gradients) per layer,
  // and the forward packs of the head and trunk layers
  bf16_t* packs = nullptr;
  int64_t pT_a[kMaxLevels] = {}, pT_b[kMaxLevels] = {}, pT_c[kMaxLevels] = {}, pT_d[kMaxLevels] = {},
          pT_up[kMaxLevels] = {}, pT_head = 0, pT_tr[9] = {}, pF_head = 0, pF_tr[9] = {};
  int kT_a[kMaxLevels] = {}, kT_b[kMaxLevels] = {}, kT_c[kMaxLevels] = {}, kT_d[kMaxLevels] = {},
      kT_up[kMaxLevels] = {}, kT_head = 0, kT_tr[9] = {}, kF_head = 0, kF_tr[9] = {};
  // FP32 / FP64 vectors and partial sums
  float* f32 = nullptr;  // y, Ay, res, gAy: [4][nb][N]
  float* part = nullptr;
  int64_t part_len = 0;
  double* dpart = nullptr;  // [nb][kRedBlocks] input-scale partials, then loss partials and the loss value
  // generated right-hand sides (R == NULL)
  GenWs gen;
  float* d_R = nullptr;  // [nb][N]
  double* gpart = nullptr;  // [kRedBlocks] partial sums of the squared gradient (clipping, SAM)
  float* w_save = nullptr;  // [np] weights kept during a sharpness-aware step
  double* sup = nullptr;    // supervised loss: [nb][5][kSupParts] partial sums, then [nb] sample losses
  int sup_nb = 0;
};

constexpr int kSupParts = 64;

static int pad8(int c) { return (c + 7) / 8 * 8; }

void net_train_free(ppe_net* n) {
  TrainState* t = n->train;
  if (!t) return;
  dev_free(t->d_lv);
  dev_free(t->d_coefs);
  dev_free((void*)t->d_masks);
  gen_free(t->gen);
  dev_free(t->d_R);
  dev_free(t->gpart);
  dev_free(t->w_save);
  dev_free(t->sup);
  dev_free(t->act);
  dev_free(t->grad);
  dev_free(t->eta);
  dev_free(t->packs);
  dev_free(t->f32);
  dev_free(t->part);
  dev_free(t->dpart);
  delete t;
  n->train = nullptr;
}

static ppe_status train_state(ppe_net* n, int nb, int nx, int ny) {
  TrainState* t = n->train;
  if (t && t->nb == nb && t->nx == nx && t->ny == ny) return PPE_OK;
  net_train_free(n);
  n->train = t = new TrainState();
  const ppe_net_config& cfg = n->cfg;
  const int L = cfg.levels, P = cfg.basis, TWd = cfg.trunk_width;
  t->nb = nb;
  t->nx = nx;
  t->ny = ny;
  t->L = L;
  for (int l = 0; l < L; ++l) {
    t->H[l] = ny >> l;
    t->W[l] = nx >> l;
  }
  auto ch = [&](int l) { return cfg.base_channels << l; };
  auto hw = [&](int l) { return (int64_t)t->H[l] * t->W[l]; };
  int64_t ao = 0, go = 0, eo = 0;
  auto A = [&](int64_t& o, int l, int pitch) {
    const int64_t r = o;
    o += hw(l) * pitch * nb;
    o = (o + 127) / 128 * 128;
    return r;
  };
  for (int l = 0; l < L; ++l) {
    t->p_in[l] = n->enc_a[l].cin8;
    t->o_in[l] = A(ao, l, t->p_in[l]);
    t->o_a[l] = A(ao, l, ch(l));
    t->g_in[l] = A(go, l, t->p_in[l]);
    t->g_a[l] = A(go, l, ch(l));
    if (l < L - 1) {
      t->p_cat[l] = n->dec_c[l].cin8;
      t->o_cat[l] = A(ao, l, t->p_cat[l]);
      t->o_c[l] = A(ao, l, ch(l));
      t->o_d[l] = A(ao, l, ch(l));
      t->g_cat[l] = A(go, l, t->p_cat[l]);
      t->g_c[l] = A(go, l, ch(l));
      t->g_d[l] = A(go, l, ch(l));
      t->g_E[l] = A(go, l, ch(l));
      t->g_Uc[l] = A(go, l + 1, ch(l));
    } else {
      t->o_bot = A(ao, l, ch(l));
      t->g_bot = A(go, l, ch(l));
    }
    if (cfg.use_eta) {  // per-sample maps: one weight per pixel, or one per input channel
      auto ep = [&](const MConvL& m) { return cfg.use_eta == 2 ? 1 : m.cin8; };
      t->e_a[l] = A(eo, l, ep(n->enc_a[l]));
      t->e_b[l] = A(eo, l, ep(n->enc_b[l]));
      if (l < L - 1) {
        t->e_c[l] = A(eo, l, ep(n->dec_c[l]));
        t->e_d[l] = A(eo, l, ep(n->dec_d[l]));
      }
    }
  }
  t->o_B = A(ao, 0, P);
  t->o_T = A(ao, 0, P);
  t->o_t0 = A(ao, 0, 8);
  for (int k = 0; k < cfg.trunk_hidden; ++k) t->o_h[k] = A(ao, 0, TWd);
  t->g_B = A(go, 0, P);
  t->g_T = A(go, 0, P);
  for (int k = 0; k < cfg.trunk_hidden; ++k) t->g_h[k] = A(go, 0, TWd);
  // packed weights of this step
  int64_t po = 0;
  auto pk = [&](int rows, int kp) {
    const int64_t r = po;
    po += (int64_t)rows * kp;
    return r;
  };
  for (int l = 0; l < L; ++l) {
    const MConvL& a = n->enc_a[l];
    const MConvL& b = n->enc_b[l];
    t->kT_a[l] = conv_packed_k(9, a.cout);
    t->pT_a[l] = pk(a.cin8, t->kT_a[l]);
    t->kT_b[l] = conv_packed_k(9, b.cout);
    t->pT_b[l] = pk(b.cin8, t->kT_b[l]);
    if (l < L - 1) {
      const MConvL& c = n->dec_c[l];
      const MConvL& d = n->dec_d[l];
      const UpL& u = n->up[l];
      t->kT_c[l] = conv_packed_k(9, c.cout);
      t->pT_c[l] = pk(c.cin8, t->kT_c[l]);
      t->kT_d[l] = conv_packed_k(9, d.cout);
      t->pT_d[l] = pk(d.cin8, t->kT_d[l]);
      t->kT_up[l] = conv_packed_k(1, u.cout);
      t->pT_up[l] = pk(u.cin, t->kT_up[l]);
    }
  }
  t->kF_head = conv_packed_k(1, cfg.base_channels);
  t->pF_head = pk(P, t->kF_head);
  t->kT_head = conv_packed_k(1, P);
  t->pT_head = pk(cfg.base_channels, t->kT_head);
  for (int k = 0; k <= cfg.trunk_hidden; ++k) {
    const int cin8 = k == 0 ? 8 : TWd;
    const int cout = k == cfg.trunk_hidden ? P : TWd;
    t->kF_tr[k] = conv_packed_k(1, cin8);
    t->pF_tr[k] = pk(cout, t->kF_tr[k]);
    t->kT_tr[k] = conv_packed_k(1, cout);
    t->pT_tr[k] = pk(cin8, t->kT_tr[k]);
  }
  const int64_t N = (int64_t)nx * ny;
  t->part_len = (int64_t)16 << 20;  // floats
  t->act = (bf16_t*)dev_alloc(ao * sizeof(bf16_t));
  t->grad = (bf16_t*)dev_alloc(go * sizeof(bf16_t));
  t->eta = cfg.use_eta ? (bf16_t*)dev_alloc(eo * sizeof(bf16_t)) : nullptr;
  t->packs = (bf16_t*)dev_alloc(po * sizeof(bf16_t));
  t->f32 = (float*)dev_alloc(4 * N * nb * sizeof(float));
  t->part = (float*)dev_alloc(t->part_len * sizeof(float));
  t->dpart = (double*)dev_alloc(((size_t)kRedBlocks * (nb + 1) + 8) * sizeof(double));
  t->d_coefs = (Coef*)dev_alloc(nb * sizeof(Coef));
  t->d_masks = (const uint8_t**)dev_alloc(nb * sizeof(void*));
  if (!t->act || !t->grad || (cfg.use_eta && !t->eta) || !t->packs || !t->f32 || !t->part || !t->dpart ||
      !t->d_coefs || !t->d_masks)
    return set_error(PPE_ERR_HIP, "allocation of the training workspace failed");
  HIPCHK(hipMemset(t->act, 0, ao * sizeof(bf16_t)));
  HIPCHK(hipMemset(t->grad, 0, go * sizeof(bf16_t)));
  return PPE_OK;
}

static int wgrad_splits(int cout, int cin8, int taps, int64_t tiles, int64_t cap) {
  const int tb = taps == 1 ? 128 : 32;  // channel tile of the 1x1 / 3x3 weight-gradient kernels
  const int64_t blocks = (int64_t)((cout + tb - 1) / tb) * ((cin8 + tb - 1) / tb);
  int64_t ns = std::max<int64_t>(1, 1024 / blocks);
  ns = std::min<int64_t>(ns, tiles);
  ns = std::min<int64_t>(ns, cap / ((int64_t)cout * cin8 * taps));
  return (int)std::max<int64_t>(ns, 1);
}

}  // namespace ppe

using namespace ppe;

extern "C" ppe_status ppe_net_train_step(ppe_net* n, int32_t nb, ppe_problem* const* problems, const float* R,
                                         const double* target, const ppe_train_opts* opts, float* loss_out,
                                         float* grad_out, hipStream_t s) {
  if (!n || !problems || !opts) return set_error(PPE_ERR_INVALID_ARG, "net, problems or opts NULL");
  if (opts->loss_kind != PPE_LOSS_RESIDUAL && opts->loss_kind != PPE_LOSS_SUPERVISED &&
      opts->loss_kind != PPE_LOSS_ANORM)
    return set_error(PPE_ERR_INVALID_ARG, "loss_kind %d", opts->loss_kind);
  if (opts->loss_kind != PPE_LOSS_RESIDUAL && (!R || !target))
    return set_error(PPE_ERR_INVALID_ARG, "the supervised and A-norm losses need an explicit batch R and its target");
  if (opts->loss_kind == PPE_LOSS_RESIDUAL && target)
    return set_error(PPE_ERR_INVALID_ARG, "target is given but the loss is the residual loss");
  if (nb < 1 || nb > 4096) return set_error(PPE_ERR_INVALID_ARG, "nb must lie in [1, 4096]");
  for (int i = 0; i < nb; ++i)
    if (problems[i] && problems[i]->mask_mode == PPE_MASK_SOLID) return reject_solid(problems[i], "ppe_net_train_step");
  if (!R) {
    ppe_status sg = check_gen_opts(*opts);
    if (sg != PPE_OK) return sg;
  }
  if (!(opts->clip_norm >= 0.f) || !std::isfinite(opts->clip_norm))
    return set_error(PPE_ERR_INVALID_ARG, "clip_norm must be finite and >= 0");
  if (!(opts->sam_rho >= 0.f) || !std::isfinite(opts->sam_rho))
    return set_error(PPE_ERR_INVALID_ARG, "sam_rho must be finite and >= 0");
  for (int i = 0; i < nb; ++i) {
    if (!problems[i]) return set_error(PPE_ERR_INVALID_ARG, "problems[%d] is NULL", i);
    if (problems[i]->nx != problems[0]->nx || problems[i]->ny != problems[0]->ny)
      return set_error(PPE_ERR_SHAPE, "all training grids must have one size");
    ppe_status st = check_net_grid(problems[i], n);
    if (st != PPE_OK) return st;
  }
  const ppe_net_config& cfg = n->cfg;
  const int nx = problems[0]->nx, ny = problems[0]->ny, L = cfg.levels, P = cfg.basis, TWd = cfg.trunk_width;
  const int TH = cfg.trunk_hidden, HID = cfg.phi_hidden, C0 = cfg.base_channels;
  if (cfg.use_eta == 1) {
    auto fits = [&](const MConvL& m) { return m.cin == 0 || eta_bwd_fits(m.cin, m.cin8, HID); };
    for (int l = 0; l < L; ++l) {
      const bool ok = fits(n->enc_a[l]) && fits(n->enc_b[l]) && (l > L - 2 || (fits(n->dec_c[l]) && fits(n->dec_d[l])));
      if (!ok)
        return set_error(PPE_ERR_INVALID_ARG,
                         "level %d is too wide for the training kernels (inputs x phi_hidden must fit the LDS)", l);
    }
  }
  const int64_t N = (int64_t)nx * ny;
  if (N * nb >= (int64_t)1 << 31)
    return set_error(PPE_ERR_INVALID_ARG, "nb x cells must stay below 2^31 (got %lld)", (long long)(N * nb));
  ppe_status st = train_state(n, nb, nx, ny);
  if (st != PPE_OK) return st;
  TrainState* t = n->train;
  const bool supervised = opts->loss_kind == PPE_LOSS_SUPERVISED;
  const bool anorm = opts->loss_kind == PPE_LOSS_ANORM;
  if ((supervised || anorm) && t->sup_nb < nb) {
    dev_free(t->sup);
    t->sup = (double*)dev_alloc(sizeof(double) * ((size_t)nb * 5 * kSupParts + nb));
    t->sup_nb = t->sup ? nb : 0;
    if (!t->sup) return set_error(PPE_ERR_HIP, "allocation of the supervised-loss sums failed");
  }
  if (!R) {
    if (!t->d_R) t->d_R = (float*)dev_alloc(sizeof(float) * N * nb);
    if (!t->d_R) return set_error(PPE_ERR_HIP, "allocation of the generated batch failed");
    st = generate_rhs(t->gen, nb, problems, *opts, t->d_R, s);
    if (st != PPE_OK) return st;
    R = t->d_R;
  }
  auto ch = [&](int l) { return C0 << l; };
  auto hw = [&](int l) { return (int64_t)t->H[l] * t->W[l]; };

  // per-sample grid data
  {
    std::vector<float> all, one;
    int64_t off[kMaxLevels], toff = 0;
    for (int i = 0; i < nb; ++i) {
      grid_block(problems[i], L, one, off, &toff);
      if (i == 0) {
        t->lv_stride = (int64_t)one.size();
        std::copy(off, off + L, t->lv_off);
        t->tin_off = toff;
        all.reserve((size_t)t->lv_stride * nb);
      }
      all.insert(all.end(), one.begin(), one.end());
    }
    dev_free(t->d_lv);
    t->d_lv = (float*)dev_alloc(all.size() * sizeof(float));
    if (!t->d_lv) return set_error(PPE_ERR_HIP, "allocation of grid arrays failed");
    HIPCHK(hipMemcpyAsync(t->d_lv, all.data(), all.size() * sizeof(float), hipMemcpyHostToDevice, s));
    std::vector<Coef> cs(nb);
    std::vector<const uint8_t*> ms(nb);
    for (int i = 0; i < nb; ++i) {
      cs[i] = problems[i]->coef;
      ms[i] = problems[i]->d_mask;
    }
    HIPCHK(hipMemcpyAsync(t->d_coefs, cs.data(), nb * sizeof(Coef), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync((void*)t->d_masks, ms.data(), nb * sizeof(void*), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));  // host vectors go out of scope
  }
  bf16_t* Ab = t->act;
  bf16_t* G = t->grad;
  bf16_t* E = t->eta;
  bf16_t* PK = t->packs;
  const float* W = n->d_w;
  float* dG = n->d_g;

  double* lpart = t->dpart + (size_t)kRedBlocks * nb;
  // One forward and backward pass at the current weights: the loss sum in
  // lpart[kRedBlocks] and the gradient in dG.
  const bool per_node = cfg.use_eta == 2;
  auto fwd_bwd = [&]() -> ppe_status {
    // packed weights of this step (transposed operators and the head / trunk forward)
    for (int l = 0; l < L; ++l) {
      const MConvL& a = n->enc_a[l];
      const MConvL& b = n->enc_b[l];
      launch_pack_weights_t(W + a.oW, a.cout, a.cin, a.cin8, 9, t->kT_a[l], PK + t->pT_a[l], s);
      launch_pack_weights_t(W + b.oW, b.cout, b.cin, b.cin8, 9, t->kT_b[l], PK + t->pT_b[l], s);
      if (l < L - 1) {
        const MConvL& c = n->dec_c[l];
        const MConvL& d = n->dec_d[l];
        const UpL& u = n->up[l];
        launch_pack_weights_t(W + c.oW, c.cout, c.cin, c.cin8, 9, t->kT_c[l], PK + t->pT_c[l], s);
        launch_pack_weights_t(W + d.oW, d.cout, d.cin, d.cin8, 9, t->kT_d[l], PK + t->pT_d[l], s);
        launch_pack_weights_t(W + u.oW, u.cout, u.cin, u.cin, 1, t->kT_up[l], PK + t->pT_up[l], s);
      }
    }
    launch_pack_weights(W + n->o_headW, P, C0, C0, 1, t->kF_head, PK + t->pF_head, s);
    launch_pack_weights_t(W + n->o_headW, P, C0, C0, 1, t->kT_head, PK + t->pT_head, s);
    for (int k = 0; k <= TH; ++k) {
      const int cin = k == 0 ? 2 : TWd, cin8 = k == 0 ? 8 : TWd, cout = k == TH ? P : TWd;
      launch_pack_weights(W + n->o_tW[k], cout, cin, cin8, 1, t->kF_tr[k], PK + t->pF_tr[k], s);
      launch_pack_weights_t(W + n->o_tW[k], cout, cin, cin8, 1, t->kT_tr[k], PK + t->pT_tr[k], s);
    }

    // static channels, trunk input and per-sample eta maps
    for (int l = 0; l < L; ++l) {
      const float* lvl = t->d_lv + t->lv_off[l];
      const int coff_in = cfg.use_spacing ? (l == 0 ? 2 : ch(l - 1)) : -1;
      launch_fill_static_multi(t->H[l], t->W[l], t->p_in[l], coff_in, lvl, t->lv_stride, t->d_masks, l == 0 ? 1 : -1,
                               Ab + t->o_in[l], hw(l) * t->p_in[l], nb, s);
      if (l < L - 1 && cfg.use_spacing)
        launch_fill_static_multi(t->H[l], t->W[l], t->p_cat[l], 2 * ch(l), lvl, t->lv_stride, nullptr, -1,
                                 Ab + t->o_cat[l], hw(l) * t->p_cat[l], nb, s);
    }
    launch_trunk_input(ny, nx, t->d_lv + t->tin_off, t->lv_stride, Ab + t->o_t0, nb, s);
    auto eta_fwd = [&](const MConvL& m, int64_t off) {
      const int l = m.level;
      // one weight per node: the same kernel with Phi's single output
      const int k = per_node ? 1 : m.cin, k8 = per_node ? 1 : m.cin8;
      launch_eta_multi(t->H[l], t->W[l], k, k8, HID, t->d_lv + t->lv_off[l], t->lv_stride, W + m.oW1, W + m.ob1,
                       W + m.oW2, W + m.ob2, E + off, hw(l) * k8, nb, s);
    };
    if (cfg.use_eta)
      for (int l = 0; l < L; ++l) {
        eta_fwd(n->enc_a[l], t->e_a[l]);
        eta_fwd(n->enc_b[l], t->e_b[l]);
        if (l < L - 1) {
          eta_fwd(n->dec_c[l], t->e_c[l]);
          eta_fwd(n->dec_d[l], t->e_d[l]);
        }
      }
    auto etap = [&](int64_t off) -> const bf16_t* { return cfg.use_eta ? E + off : nullptr; };
    auto geo = [&](int l, int cin8, int cout, int y_pitch, int y_off, int act) {
      ConvGeo g{};
      g.H = t->H[l];
      g.W = t->W[l];
      g.cin8 = cin8;
      g.x_pitch = cin8;
      g.c1 = cin8;
      g.x1_pitch = 0;
      g.x1 = nullptr;
      g.x1_bstride = 0;
      g.cout = cout;
      g.y_pitch = y_pitch;
      g.y_off = y_off;
      g.x_bstride = hw(l) * cin8;
      g.y_bstride = hw(l) * y_pitch;
      g.e_bstride = hw(l) * (per_node ? 1 : cin8);
      g.act = act;
      g.eta_node = per_node;
      return g;
    };

    // ---- forward, saving activations ----
    float* y = t->f32;
    float* Ay = y + N * nb;
    float* res = Ay + N * nb;
    float* gAy = res + N * nb;
    launch_input_pack(R, N, nb, t->dpart, Ab + t->o_in[0], t->p_in[0], N * t->p_in[0], s);
    for (int l = 0; l < L; ++l) {
      if (l > 0)
        launch_pool2(t->H[l], t->W[l], ch(l - 1), Ab + t->o_cat[l - 1], t->p_cat[l - 1], ch(l - 1),
                     4 * hw(l) * t->p_cat[l - 1], Ab + t->o_in[l], t->p_in[l], hw(l) * t->p_in[l], nb, s);
      const MConvL& ma = n->enc_a[l];
      const MConvL& mb = n->enc_b[l];
      launch_conv(9, false, geo(l, ma.cin8, ma.cout, ch(l), 0, 1), nb, Ab + t->o_in[l], etap(t->e_a[l]),
                  n->d_pack + ma.opack, ma.kp, W + ma.ob, Ab + t->o_a[l], s);
      if (l < L - 1)
        launch_conv(9, false, geo(l, mb.cin8, mb.cout, t->p_cat[l], ch(l), 1), nb, Ab + t->o_a[l], etap(t->e_b[l]),
                    n->d_pack + mb.opack, mb.kp, W + mb.ob, Ab + t->o_cat[l], s);
      else
        launch_conv(9, false, geo(l, mb.cin8, mb.cout, ch(l), 0, 1), nb, Ab + t->o_a[l], etap(t->e_b[l]),
                    n->d_pack + mb.opack, mb.kp, W + mb.ob, Ab + t->o_bot, s);
    }
    for (int l = L - 2; l >= 0; --l) {
      const UpL& u = n->up[l];
      const bf16_t* src = (l == L - 2) ? Ab + t->o_bot : Ab + t->o_d[l + 1];
      ConvGeo gu = geo(l + 1, u.cin, u.cout, t->p_cat[l], 0, 0);
      gu.y_bstride = hw(l) * t->p_cat[l];
      launch_conv(1, true, gu, nb, src, nullptr, n->d_pack + u.opack, u.kp, W + u.ob, Ab + t->o_cat[l], s);
      const MConvL& mc = n->dec_c[l];
      const MConvL& md = n->dec_d[l];
      launch_conv(9, false, geo(l, mc.cin8, mc.cout, ch(l), 0, 1), nb, Ab + t->o_cat[l], etap(t->e_c[l]),
                  n->d_pack + mc.opack, mc.kp, W + mc.ob, Ab + t->o_c[l], s);
      launch_conv(9, false, geo(l, md.cin8, md.cout, ch(l), 0, 1), nb, Ab + t->o_c[l], etap(t->e_d[l]),
                  n->d_pack + md.opack, md.kp, W + md.ob, Ab + t->o_d[l], s);
    }
    // head B = Wh D0 + bh and trunk T (BF16 MFMA, tanh hidden layers), then y
    launch_conv(1, false, geo(0, C0, P, P, 0, 0), nb, Ab + t->o_d[0], nullptr, PK + t->pF_head, t->kF_head,
                W + n->o_headb, Ab + t->o_B, s);
    for (int k = 0; k <= TH; ++k) {
      const int cin8 = k == 0 ? 8 : TWd, cout = k == TH ? P : TWd;
      const bf16_t* src = k == 0 ? Ab + t->o_t0 : Ab + t->o_h[k - 1];
      bf16_t* dst = k == TH ? Ab + t->o_T : Ab + t->o_h[k];
      launch_conv(1, false, geo(0, cin8, cout, cout, 0, k == TH ? 0 : 2), nb, src, nullptr, PK + t->pF_tr[k],
                  t->kF_tr[k], W + n->o_tb[k], dst, s);
    }
    launch_don_fwd(N * nb, P, Ab + t->o_B, Ab + t->o_T, W + n->o_gamma, y, s);

    float dscale = 1.f;
    if (supervised) {
      // ---- supervised loss: dL/dy straight into gAy ----
      launch_sup_loss(N, nb, y, target, t->sup, kSupParts, gAy, t->sup + (size_t)nb * 5 * kSupParts, s);
      launch_sum_parts(t->sup + (size_t)nb * 5 * kSupParts, nb, 1.0 / nb, lpart + kRedBlocks, s);
    } else if (anorm) {
      // ---- A-norm loss: dL/dy = c_R R + c_A A y per sample, into gAy ----
      launch_apply_multi(t->d_coefs, nx, ny, nb, y, Ay, s);
      launch_anorm_loss(N, nb, y, Ay, R, target, t->sup, kSupParts, gAy, t->sup + (size_t)nb * 5 * kSupParts, s);
      launch_sum_parts(t->sup + (size_t)nb * 5 * kSupParts, nb, 1.0 / nb, lpart + kRedBlocks, s);
    } else {
      // ---- loss (Eq. 19): res = R - A y, L = mean(res^2); dL/dy = -2/(nb N) A res ----
      launch_apply_multi(t->d_coefs, nx, ny, nb, y, Ay, s);
      launch_loss(N * nb, R, Ay, res, lpart, kRedBlocks, s);
      launch_sum_parts(lpart, kRedBlocks, 1.0 / ((double)N * nb), lpart + kRedBlocks, s);
      launch_apply_multi(t->d_coefs, nx, ny, nb, res, gAy, s);
      dscale = (float)(-2.0 / ((double)N * nb));
    }

    // ---- backward ----
    HIPCHK(hipMemsetAsync(dG, 0, n->np * sizeof(float), s));
    float* part = t->part;
    const int64_t cap = t->part_len;
    auto tiles_of = [&](int l) {
      return (int64_t)((t->W[l] + 15) / 16) * ((t->H[l] + 7) / 8) * nb;
    };
    auto wgrad = [&](int taps, int l, const bf16_t* dp, int dp_pitch, int cout, const bf16_t* x, int cin8, int cin,
                     const bf16_t* eta, int64_t oW) {
      WgradGeo g;
      g.H = t->H[l];
      g.W = t->W[l];
      g.nb = nb;
      g.cin8 = cin8;
      g.cin = cin;
      g.cout = cout;
      g.dp_pitch = dp_pitch;
      g.x_bstride = hw(l) * cin8;
      g.dp_bstride = hw(l) * dp_pitch;
      g.e_bstride = hw(l) * (per_node ? 1 : cin8);
      g.eta_node = per_node;
      const int ns = wgrad_splits(cout, cin8, taps, tiles_of(l), cap);
      launch_wgrad(taps, g, dp, x, eta, part, ns, s);
      launch_reduce_rows(part, ns, (int64_t)cout * cin * taps, 1.f, dG + oW, s);
    };
    auto bias = [&](int l, const bf16_t* d, int pitch, int C, int64_t ob) {
      launch_bias_grad(d, hw(l) * nb, pitch, 0, C, part, 1024, s);
      launch_reduce_rows(part, 1024, C, 1.f, dG + ob, s);
    };
    auto dgrad = [&](int taps, int l, const bf16_t* dp, int cout_fwd, int64_t pT, int kT, int rows, bf16_t* out) {
      ConvGeo g = geo(l, cout_fwd, rows, rows, 0, 0);
      launch_conv(taps, false, g, nb, dp, nullptr, PK + pT, kT, nullptr, out, s);
    };
    auto eta_bwd = [&](const MConvL& m, const bf16_t* x, int64_t eoff, bf16_t* dxb) {
      if (!cfg.use_eta) return;
      const int l = m.level;
      const int len = per_node ? eta_bwd_node_len(HID) : eta_bwd_len(m.cin, HID);
      // partial rows: up to 2048, as many as the partials buffer holds
      int np = (int)std::min<int64_t>(2048, cap / len);
      if (per_node) {
        np = (int)std::min<int64_t>(np, (hw(l) * nb + 255) / 256);
        launch_eta_bwd_node(t->H[l], t->W[l], m.cin8, HID, nb, t->d_lv + t->lv_off[l], t->lv_stride, W + m.oW1,
                            W + m.ob1, W + m.oW2, W + m.ob2, x, E + eoff, dxb, part, np, s);
      } else {
        launch_eta_bwd(t->H[l], t->W[l], m.cin, m.cin8, HID, nb, t->d_lv + t->lv_off[l], t->lv_stride, W + m.oW1,
                       W + m.ob1, W + m.oW2, W + m.ob2, x, E + eoff, hw(l) * m.cin8, dxb, part, np, s);
      }
      launch_reduce_rows(part, np, len, 1.f, dG + m.oW1, s);
    };
    // DeepONet contraction, head and trunk
    launch_don_bwd(N * nb, P, Ab + t->o_B, Ab + t->o_T, W + n->o_gamma, gAy, dscale, G + t->g_B, G + t->g_T, part,
                   2048, s);
    launch_reduce_rows(part, 2048, 1, 1.f, dG + n->o_gamma, s);
    wgrad(1, 0, G + t->g_B, P, P, Ab + t->o_d[0], C0, C0, nullptr, n->o_headW);
    bias(0, G + t->g_B, P, P, n->o_headb);
    dgrad(1, 0, G + t->g_B, P, t->pT_head, t->kT_head, C0, G + t->g_d[0]);
    for (int k = TH; k >= 0; --k) {
      const int cin8 = k == 0 ? 8 : TWd, cin = k == 0 ? 2 : TWd, cout = k == TH ? P : TWd;
      bf16_t* dk = k == TH ? G + t->g_T : G + t->g_h[k];
      if (k < TH) launch_act_bwd(dk, cout, Ab + t->o_h[k], cout, 0, cout, N * nb, 2, s);
      const bf16_t* xin = k == 0 ? Ab + t->o_t0 : Ab + t->o_h[k - 1];
      wgrad(1, 0, dk, cout, cout, xin, cin8, cin, nullptr, n->o_tW[k]);
      bias(0, dk, cout, cout, n->o_tb[k]);
      if (k > 0) dgrad(1, 0, dk, cout, t->pT_tr[k], t->kT_tr[k], cin8, G + t->g_h[k - 1]);
    }
    // decoder, finest level first
    for (int l = 0; l <= L - 2; ++l) {
      const MConvL& md = n->dec_d[l];
      const MConvL& mc = n->dec_c[l];
      const UpL& u = n->up[l];
      bf16_t* dD = G + t->g_d[l];
      launch_act_bwd(dD, ch(l), Ab + t->o_d[l], ch(l), 0, ch(l), hw(l) * nb, 1, s);
      wgrad(9, l, dD, ch(l), ch(l), Ab + t->o_c[l], md.cin8, md.cin, etap(t->e_d[l]), md.oW);
      bias(l, dD, ch(l), ch(l), md.ob);
      dgrad(9, l, dD, ch(l), t->pT_d[l], t->kT_d[l], md.cin8, G + t->g_c[l]);
      eta_bwd(md, Ab + t->o_c[l], t->e_d[l], G + t->g_c[l]);
      launch_act_bwd(G + t->g_c[l], ch(l), Ab + t->o_c[l], ch(l), 0, ch(l), hw(l) * nb, 1, s);
      wgrad(9, l, G + t->g_c[l], ch(l), ch(l), Ab + t->o_cat[l], mc.cin8, mc.cin, etap(t->e_c[l]), mc.oW);
      bias(l, G + t->g_c[l], ch(l), ch(l), mc.ob);
      dgrad(9, l, G + t->g_c[l], ch(l), t->pT_c[l], t->kT_c[l], mc.cin8, G + t->g_cat[l]);
      eta_bwd(mc, Ab + t->o_cat[l], t->e_c[l], G + t->g_cat[l]);
      launch_copy_ch(G + t->g_cat[l], t->p_cat[l], ch(l), G + t->g_E[l], ch(l), ch(l), hw(l) * nb, 0, s);
      launch_up_bwd(t->H[l + 1], t->W[l + 1], ch(l), G + t->g_cat[l], t->p_cat[l], hw(l) * t->p_cat[l],
                    G + t->g_Uc[l], hw(l + 1) * ch(l), nb, s);
      const bf16_t* src = (l == L - 2) ? Ab + t->o_bot : Ab + t->o_d[l + 1];
      wgrad(1, l + 1, G + t->g_Uc[l], ch(l), ch(l), src, u.cin, u.cin, nullptr, u.oW);
      bias(l + 1, G + t->g_Uc[l], ch(l), ch(l), u.ob);
      bf16_t* dnext = (l == L - 2) ? G + t->g_bot : G + t->g_d[l + 1];
      dgrad(1, l + 1, G + t->g_Uc[l], ch(l), t->pT_up[l], t->kT_up[l], u.cin, dnext);
    }
    // encoder, coarsest level first
    for (int l = L - 1; l >= 0; --l) {
      const MConvL& mb = n->enc_b[l];
      const MConvL& ma = n->enc_a[l];
      bf16_t* dE = (l == L - 1) ? G + t->g_bot : G + t->g_E[l];
      if (l == L - 1)
        launch_act_bwd(dE, ch(l), Ab + t->o_bot, ch(l), 0, ch(l), hw(l) * nb, 1, s);
      else
        launch_act_bwd(dE, ch(l), Ab + t->o_cat[l], t->p_cat[l], ch(l), ch(l), hw(l) * nb, 1, s);
      wgrad(9, l, dE, ch(l), ch(l), Ab + t->o_a[l], mb.cin8, mb.cin, etap(t->e_b[l]), mb.oW);
      bias(l, dE, ch(l), ch(l), mb.ob);
      dgrad(9, l, dE, ch(l), t->pT_b[l], t->kT_b[l], mb.cin8, G + t->g_a[l]);
      eta_bwd(mb, Ab + t->o_a[l], t->e_b[l], G + t->g_a[l]);
      launch_act_bwd(G + t->g_a[l], ch(l), Ab + t->o_a[l], ch(l), 0, ch(l), hw(l) * nb, 1, s);
      wgrad(9, l, G + t->g_a[l], ch(l), ch(l), Ab + t->o_in[l], ma.cin8, ma.cin, etap(t->e_a[l]), ma.oW);
      bias(l, G + t->g_a[l], ch(l), ch(l), ma.ob);
      if (cfg.use_eta || l > 0) {
        dgrad(9, l, G + t->g_a[l], ch(l), t->pT_a[l], t->kT_a[l], ma.cin8, G + t->g_in[l]);
        eta_bwd(ma, Ab + t->o_in[l], t->e_a[l], G + t->g_in[l]);
      }
      if (l > 0)
        launch_pool_bwd(t->H[l], t->W[l], ch(l - 1), G + t->g_in[l], t->p_in[l], hw(l) * t->p_in[l],
                        G + t->g_E[l - 1], hw(l - 1) * ch(l - 1), nb, s);
    }
    HIPCHK(hipGetLastError());
    return PPE_OK;
  };

  st = fwd_bwd();
  if (st != PPE_OK) return st;
  double loss = 0.0;
  HIPCHK(hipMemcpyAsync(&loss, lpart + kRedBlocks, sizeof(double), hipMemcpyDeviceToHost, s));
  if (opts->sam_rho > 0.f) {
    // Sharpness-aware step: the gradient is taken again at w + rho g / |g|
    // (|g| in FP64, fixed order), and Adam updates w with that gradient.
    if (!t->gpart) t->gpart = (double*)dev_alloc(sizeof(double) * kRedBlocks);
    if (!t->w_save) t->w_save = (float*)dev_alloc(sizeof(float) * n->np);
    if (!t->gpart || !t->w_save) return set_error(PPE_ERR_HIP, "allocation of the SAM buffers failed");
    launch_sumsq(dG, n->np, 1, t->gpart, s);
    HIPCHK(hipMemcpyAsync(t->w_save, n->d_w, n->np * sizeof(float), hipMemcpyDeviceToDevice, s));
    launch_sam_perturb(n->np, n->d_w, dG, t->gpart, opts->sam_rho, s);
    st = net_refresh(n, s);
    if (st != PPE_OK) return st;
    st = fwd_bwd();
    if (st != PPE_OK) return st;
    HIPCHK(hipMemcpyAsync(n->d_w, t->w_save, n->np * sizeof(float), hipMemcpyDeviceToDevice, s));
    st = net_refresh(n, s);
    if (st != PPE_OK) return st;
  }
  if (grad_out) HIPCHK(hipMemcpyAsync(grad_out, dG, n->np * sizeof(float), hipMemcpyDeviceToHost, s));
  // ---- Adam ----
  if (opts->lr > 0.f) {
    n->step += 1;
    const float c1 = 1.f - std::pow(opts->beta1, (float)n->step);
    const float c2 = 1.f - std::pow(opts->beta2, (float)n->step);
    if (opts->clip_norm > 0.f) {
      if (!t->gpart) t->gpart = (double*)dev_alloc(sizeof(double) * kRedBlocks);
      if (!t->gpart) return set_error(PPE_ERR_HIP, "allocation of the gradient-norm partials failed");
      launch_sumsq(dG, n->np, 1, t->gpart, s);
    }
    launch_adam(n->np, n->d_w, dG, n->d_m, n->d_v, opts->lr, opts->beta1, opts->beta2, opts->eps, c1, c2, t->gpart,
                opts->clip_norm, s);
    st = net_refresh(n, s);
    if (st != PPE_OK) return st;
  }
  HIPCHK(hipStreamSynchronize(s));
  if (loss_out) *loss_out = (float)loss;
  return PPE_OK;
}
