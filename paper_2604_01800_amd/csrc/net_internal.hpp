// Host-side internals of the DeepONet: parameter layout, handle, per-grid cache.
#pragma once
#include <atomic>
#include <vector>

#include "../../include/ppe.h"
#include "net_common.hpp"
#include "net_kernels.hpp"

namespace ppe {

// One Mesh-Conv layer: offsets into the FP32 parameter vector and its packed
// BF16 weights (kp values per output channel).
struct MConvL {
  int level = 0, cin = 0, cout = 0, cin8 = 0, kp = 0;
  int phik = 0;  // outputs of the local-weight network Phi: 1 per node, or cin
  int64_t oW = 0, ob = 0, oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, opack = 0;
};

// 1x1 up-convolution C_{l+1} -> C_l of decoder level l.
struct UpL {
  int level = 0, cin = 0, cout = 0, kp = 0;
  int64_t oW = 0, ob = 0, opack = 0;
};

struct TrainState;  // training workspaces (defined with the training kernels)

}  // namespace ppe

struct ppe_net {
  ppe_net_config cfg{};
  uint64_t uid = 0;       // unique id (per-grid caches key on it)
  uint64_t version = 0;   // bumped whenever the weights change
  int64_t np = 0, npack = 0, step = 0;
  std::vector<ppe::MConvL> enc_a, enc_b, dec_c, dec_d;
  std::vector<ppe::UpL> up;
  int64_t o_headW = 0, o_headb = 0, o_gamma = 0;
  std::vector<int64_t> o_tW, o_tb;
  float *d_w = nullptr, *d_g = nullptr, *d_m = nullptr, *d_v = nullptr;  // FP32 masters, grad, Adam moments
  ppe::bf16_t* d_pack = nullptr;                                         // packed BF16 conv weights
  ppe::TrainState* train = nullptr;
};

namespace ppe {

constexpr int kMaxLevels = 6;

// Per-(grid, network, batch) constants and activation buffers of the forward.
struct NetCache {
  uint64_t net_uid = 0, version = 0;
  int nb = 0, L = 0, use_eta = 0, use_spacing = 0, c0 = 0;
  int H[kMaxLevels] = {}, W[kMaxLevels] = {};
  float* d_lv = nullptr;  // 1D level arrays and trunk inputs
  int64_t lv_off[kMaxLevels] = {}, tin_off = 0;
  bf16_t* d_eta = nullptr;
  int64_t eta_a[kMaxLevels] = {}, eta_b[kMaxLevels] = {}, eta_c[kMaxLevels] = {}, eta_d[kMaxLevels] = {};
  float* d_fold = nullptr;  // [N][c0 + 1] trunk basis with the head folded in
  int fold_pitch = 0;
  bf16_t* d_act = nullptr;
  int64_t act_elems = 0;
  // channel pitches of the level inputs and of the decoder concatenations
  // (pooled or upsampled features and skip features; the static channels
  // live in o_st, one copy shared by the batch, pitch 8)
  int p_in[kMaxLevels] = {}, p_cat[kMaxLevels] = {};
  int64_t o_in[kMaxLevels] = {}, o_a[kMaxLevels] = {}, o_cat[kMaxLevels] = {}, o_c[kMaxLevels] = {},
          o_d[kMaxLevels] = {}, o_st[kMaxLevels] = {}, o_up[kMaxLevels] = {}, o_bot = 0;
  double* d_part = nullptr;
  float* d_kpart = nullptr;  // partial sums of convolutions with a split K loop
  int64_t kpart_elems = 0;
  int8_t conv_tn[64] = {};   // tuned output channels per workgroup of forward launch k (0: the default)
};

// One layer of a grouped forward: its member table (at d_tab + off) and the
// launch parameters the members share.
struct GroupOp {
  int kind = 0;            // input scaling, convolution, output (the forward's order)
  int64_t off = 0;
  int a = 0, b = 0;        // shared channel counts and pitches
  int64_t maxn = 0;        // largest member's pixels (output)
  ConvGroupLaunch conv{};
  const bf16_t* wp = nullptr;
  int Kp = 0;
  const float* bias = nullptr;
  const float* gamma = nullptr;
};

// The forwards of several grids (one field each) as one launch per layer
// and part. The grids are packed into parts of at most kGroupCells cells (a
// larger grid is a part of its own). On 48 grids of 16 M cells in all, the
// grouped forward took 17.4 ms with parts of 2^20 cells, 15.4 with 2^21,
// 15.3 with 2^22 and 15.4 with 2^23: smaller parts add launches and their
// tails, larger ones gain nothing more.
constexpr int64_t kGroupCells = int64_t(1) << 22;
struct GroupPart {
  int n = 0;
  std::vector<GroupOp> ops;
};
struct NetGroup {
  int n = 0;
  std::vector<GroupPart> parts;
  char* d_tab = nullptr;
  std::vector<char> h_tab;  // host copy of the tables (source of the upload)
};

void net_cache_free(NetCache* c);
ppe_status net_cache_ensure(ppe_problem* p, ppe_net* n, int nb, hipStream_t s);
ppe_status net_forward(ppe_problem* p, ppe_net* n, int nb, const float* r, float* y, hipStream_t s);
// Builds the group of problems[0..n) (distinct, each with one field r[i] ->
// y[i]; skip[i] = a flag whose nonzero value makes member i's launches return
// at once, or skip = null) on stream s; the member tables are uploaded on s.
ppe_status net_group_build(int n, ppe_problem* const* probs, ppe_net* net, const float* const* r, float* const* y,
                           const int32_t* const* skip, hipStream_t s, NetGroup& G);
ppe_status net_group_forward(const NetGroup& G, hipStream_t s);
void net_group_free(NetGroup& G);
ppe_status net_refresh(ppe_net* n, hipStream_t s);
ppe_status check_net_grid(const ppe_problem* p, const ppe_net* n);
// Hybrid solves of a mixed-size batch (one solve per problem, problems
// distinct), advanced round by round in lock step on stream s.
ppe_status solve_hybrid_batch_impl(int32_t n, ppe_problem* const* problems, ppe_net* net, const float* const* f,
                                   double* const* x, const ppe_solve_opts& o, ppe_solve_stats* stats,
                                   hipStream_t s);
void net_train_free(ppe_net* n);
void grid_block(const ppe_problem* p, int L, std::vector<float>& lv, int64_t* lv_off, int64_t* tin_off);

}  // namespace ppe
