// Host-side declarations of the network kernel launchers.
#pragma once
#include <vector>

#include "net_common.hpp"

namespace ppe {

constexpr int kRedBlocks = 256;  // workgroups of the fixed-size reductions

// Offsets (into the FP32 parameter vector) of the trunk layers and the head.
struct TrunkDesc {
  int hidden, width, basis, c0, fold_pitch;
  int64_t oW[9], ob[9];  // hidden layers then the output layer
  int64_t oWh, obh;      // branch head (folded into the basis)
};

// Floats of partial-sum room that lets every small layer split its K loop.
int64_t conv_kpart_elems();
// kpart (optional, kpart_elems floats): room for FP32 partial sums, which lets
// layers with fewer workgroups than compute units split their K loop.
// tn: output channels per workgroup (32 or 64; 0: conv_default_tile).
void launch_conv(int taps, bool up, const ConvGeo& g, int nb, const bf16_t* x, const bf16_t* eta, const bf16_t* wp,
                 int Kp, const float* bias, bf16_t* y, hipStream_t s, float* kpart = nullptr,
                 int64_t kpart_elems = 0, int tn = 0);
// The default tn of a layer over nb samples.
int conv_default_tile(const ConvGeo& g, int nb);
// The 3x3 convolution of launch_conv (taps 9, no upsampling) followed by the
// DeepONet output of `of` computed in its epilogue, its own output not
// stored; bit-identical to launch_conv then launch_deeponet_out. Returns
// false, launching nothing, where the layer does not allow it (more than 32
// output channels or a tile width of 64, a K split, pooling, a coarse source).
bool launch_conv_out(const ConvGeo& g, int nb, const bf16_t* x, const bf16_t* eta, const bf16_t* wp, int Kp,
                     const float* bias, bf16_t* y, hipStream_t s, float* kpart, int64_t kpart_elems, int tn,
                     const OutFold& of);
// Whether launch_conv has a choice of tn for this layer.
bool conv_has_tile_choice(int taps, bool up, bool has_eta, const ConvGeo& g, int Kp);
// Grouped convolution (one layer of the forwards of several grids): the
// launch shape that plan_conv_group derives from the members (their g, x,
// eta, y, kpart and skip set by the caller; it fills wg0, nwt and ks). Only
// 3x3 layers and 1x1 layers without local weights are grouped
// (plan_conv_group returns false otherwise). The member table must be in
// device memory for launch_conv_group.
struct ConvGroupLaunch {
  int taps = 9, up = 0, eta = 0, tn = 32, wstat = 0, run = 1, gx = 0, cot = 0, nmem = 0, split = 0, ksum_gx = 0;
  int skinny = 0;  // small 1x1 layers: the skinny GEMM with this many 16-channel tiles (2, 4, 8), else 0
  int xu = 0;      // the members have a coarse input source
};
bool plan_conv_group(int taps, bool up, int Kp, std::vector<ConvMember>& m, int64_t kpart_elems,
                     ConvGroupLaunch& L);
void launch_conv_group(const ConvGroupLaunch& L, const ConvMember* d_mem, const bf16_t* wp, int Kp,
                       const float* bias, hipStream_t s);
void launch_input_pack_group(const PackMember* d_mem, int n, int pitch, hipStream_t s);
void launch_deeponet_out_group(const OutMember* d_mem, int n, int64_t max_npix, int c0, int fold_pitch,
                               const float* gamma, hipStream_t s);
void launch_pack_weights(const float* w, int cout, int cin, int cin8, int taps, int Kp, bf16_t* out, hipStream_t s);
// Input-gradient operator: rows = input channels (padded), K over cout_fwd.
void launch_pack_weights_t(const float* w, int cout_fwd, int cin_fwd, int rows, int taps, int Kp, bf16_t* out,
                           hipStream_t s);
void launch_eta(int H, int W, int cin, int cin8, int hid, const float* dxl, const float* dxr, const float* dyd,
                const float* dyu, const float* W1, const float* b1, const float* W2, const float* b2, bf16_t* eta,
                hipStream_t s);
void launch_trunk_fold(int H, int W, const float* xin, const float* yin, const float* params, const TrunkDesc& td,
                       float* out, hipStream_t s);
void launch_fill_static(int H, int W, int pitch, int coff, const float* hxn, const float* hyn, const uint8_t* mask,
                        int moff, bf16_t* buf, int64_t bstride, int nb, hipStream_t s);
// Per-sample partial sums of r^2 (kRedBlocks per sample, [nb][kRedBlocks]).
void launch_sumsq(const float* r, int64_t n, int nb, double* part, hipStream_t s);
void launch_input_pack(const float* r, int64_t n, int nb, double* part, bf16_t* xin, int pitch, int64_t bstride,
                       hipStream_t s);
void launch_pool2(int Ho, int Wo, int C, const bf16_t* in, int pin, int cin_off, int64_t in_bs, bf16_t* out, int pout,
                  int64_t out_bs, int nb, hipStream_t s);
void launch_deeponet_out(int64_t npix, int c0, const bf16_t* d0, int64_t d_bs, const float* fold, int fold_pitch,
                         const float* gamma, float* y, int nb, hipStream_t s);

}  // namespace ppe
