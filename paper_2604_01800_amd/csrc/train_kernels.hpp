// Host-side declarations of the training kernel launchers.
#pragma once
#include "net_common.hpp"

namespace ppe {

struct WgradGeo {
  int H, W, nb;
  int cin8;           // input pitch (channels per pixel of X and eta)
  int cin;            // real input channels (gradient rows written)
  int cout;           // output channels
  int dp_pitch;       // pitch of the output gradient
  int64_t x_bstride, dp_bstride, e_bstride;  // per-sample strides (e_bstride unused without eta)
  int eta_node;       // 1: eta holds one weight per pixel ([H][W] per sample), else one per input channel
};

void launch_wgrad(int taps, const WgradGeo& g, const bf16_t* dp, const bf16_t* x, const bf16_t* eta, float* part,
                  int nsplit, hipStream_t s);
void launch_reduce_rows(const float* part, int nparts, int64_t len, float scale, float* out, hipStream_t s);
void launch_bias_grad(const bf16_t* d, int64_t npix, int pitch, int off, int C, float* part, int nparts,
                      hipStream_t s);
void launch_act_bwd(bf16_t* d, int dpitch, const bf16_t* out, int opitch, int ooff, int C, int64_t npix, int mode,
                    hipStream_t s);
void launch_copy_ch(const bf16_t* src, int spitch, int soff, bf16_t* dst, int dpitch, int C, int64_t npix, int acc,
                    hipStream_t s);
void launch_up_bwd(int Hc, int Wc, int C, const bf16_t* fine, int fpitch, int64_t f_bs, bf16_t* coarse, int64_t c_bs,
                   int nb, hipStream_t s);
void launch_pool_bwd(int Hc, int Wc, int C, const bf16_t* dpool, int ppitch, int64_t p_bs, bf16_t* dE, int64_t e_bs,
                     int nb, hipStream_t s);
void launch_eta_multi(int H, int W, int cin, int cin8, int hid, const float* lv, int64_t lv_stride, const float* W1,
                      const float* b1, const float* W2, const float* b2, bf16_t* eta, int64_t e_bs, int nb,
                      hipStream_t s);
int eta_bwd_len(int cin, int hid);
// Whether the local-weight backward handles a layer of cin inputs (pitch cin8)
// and hid hidden units: cin8 <= 1024 and its LDS rows fit the device.
bool eta_bwd_fits(int cin, int cin8, int hid);
void launch_eta_bwd(int H, int W, int cin, int cin8, int hid, int nb, const float* lv, int64_t lv_stride,
                    const float* W1, const float* b1, const float* W2, const float* b2, const bf16_t* x,
                    const bf16_t* eta, int64_t e_bs, bf16_t* dxb, float* part, int nparts, hipStream_t s);
void launch_fill_static_multi(int H, int W, int pitch, int coff, const float* lv, int64_t lv_stride,
                              const uint8_t* const* masks, int moff, bf16_t* buf, int64_t bstride, int nb,
                              hipStream_t s);
void launch_trunk_input(int H, int W, const float* tin, int64_t t_stride, bf16_t* out, int nb, hipStream_t s);
void launch_don_fwd(int64_t n, int P, const bf16_t* B, const bf16_t* T, const float* gamma, float* y, hipStream_t s);
void launch_don_bwd(int64_t n, int P, const bf16_t* B, const bf16_t* T, const float* gamma, const float* g,
                    float scale, bf16_t* dB, bf16_t* dT, float* part, int nparts, hipStream_t s);
void launch_loss(int64_t n, const float* R, const float* Ay, float* res, double* part, int nparts, hipStream_t s);
void launch_sum_parts(const double* part, int n, double scale, double* out, hipStream_t s);
// Supervised loss (scale- and shift-invariant misfit of y against the FP64
// targets e): per-sample losses into lsamp [nb] and dL/dy (batch mean) into
// dy; part holds [nb][5][nparts] partial sums.
int eta_bwd_node_len(int hid);
void launch_eta_bwd_node(int H, int W, int cin8, int hid, int nb, const float* lv, int64_t lv_stride,
                         const float* W1, const float* b1, const float* W2, const float* b2, const bf16_t* x,
                         const bf16_t* eta, bf16_t* dxb, float* part, int nparts, hipStream_t s);
void launch_anorm_loss(int64_t N, int nb, const float* y, const float* Ay, const float* R, const double* e,
                       double* part, int nparts, float* dy, double* lsamp, hipStream_t s);
void launch_sup_loss(int64_t N, int nb, const float* y, const double* e, double* part, int nparts, float* dy,
                     double* lsamp, hipStream_t s);
// Adam step; clip > 0 scales the gradient to norm <= clip first, with ||g||^2
// from the kRedBlocks partials in gpart (launch_sumsq on g).
void launch_sam_perturb(int64_t n, float* w, const float* g, const double* gpart, float rho, hipStream_t s);
void launch_adam(int64_t n, float* w, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                 float c1, float c2, const double* gpart, float clip, hipStream_t s);

}  // namespace ppe
