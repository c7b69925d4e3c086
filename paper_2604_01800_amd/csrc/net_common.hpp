// Device-side definitions shared by the network kernels (BF16 MFMA path).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ppe {

typedef uint16_t bf16_t;  // BF16 stored as raw bits
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// Round-to-nearest-even FP32 -> BF16 (NaN kept quiet): the hardware
// conversion (v_cvt_pk_bf16_f32) in device code, the same rounding in
// software on the host.
__host__ __device__ __forceinline__ bf16_t f2bf(float f) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_bit_cast(bf16_t, (__bf16)f);
#else
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (bf16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
#endif
}

__host__ __device__ __forceinline__ float bf2f(bf16_t h) {
  return __builtin_bit_cast(float, (uint32_t)h << 16);
}

// exp and tanh where the result is stored in BF16 or feeds a network
// gradient: the hardware exponential and reciprocal, relative error about
// 1e-6 (absolute for tanh near 0), far below BF16's 2^-8 step. tanh uses the
// identity tanh x = sign(x) (1 - e^{-2|x|}) / (1 + e^{-2|x|}).
__device__ __forceinline__ float exp_nn(float x) { return __expf(x); }
__device__ __forceinline__ float tanh_nn(float x) {
  const float t = __expf(-2.f * fabsf(x));
  return copysignf((1.f - t) * __builtin_amdgcn_rcpf(1.f + t), x);
}

constexpr int kConvTH = 8;   // conv pixel tile: 8 rows x 16 columns
constexpr int kConvTW = 16;
constexpr int kConvCK = 32;  // input channels staged per LDS chunk

// Geometry of one MConv / conv layer as the kernels see it.
struct ConvGeo {
  int H, W;          // pixels of the layer's level
  int cin8;          // input channels read (multiple of 8)
  int x_pitch;       // channels per pixel of the input buffer
  int c1;            // input channels [0, c1) come from the input buffer, [c1, cin8) from x1
  int x1_pitch;      // channels per pixel of x1
  const bf16_t* x1;    // second input buffer (channels c1 .. cin8-1), or null when c1 = cin8
  int64_t x1_bstride;  // elements between samples of x1 (0 = shared by the batch)
  // optional coarse source: input channels [0, cu) come from xu, a buffer at
  // half the resolution (pixel (y, x) reads (y / 2, x / 2): the nearest
  // upsampling of its values), pitch xu_pitch; cu a multiple of 32, cu <= c1
  const bf16_t* xu;
  int cu;
  int xu_pitch;
  int64_t xu_bstride;
  int cout;          // output channels
  int y_pitch;       // output buffer pitch (channels per pixel)
  int y_off;         // first output channel in that buffer
  int64_t x_bstride; // elements between samples of the input
  int64_t y_bstride; // elements between samples of the output
  int64_t e_bstride; // elements between samples of eta (0 = shared by the batch)
  int act;          // epilogue activation: 0 none, 1 ReLU, 2 tanh
  int eta_node;     // 1: eta holds one weight per pixel ([H][W]), else one per input channel (pitch cin8)
  // optional 2x2 average pooling of the output into the next level (H/2 x
  // W/2 pixels, pitch pool_pitch, output channel co at channel co; H and W
  // even; not with the upsampled output): null, or the pooled buffer
  bf16_t* pool_y;
  int pool_pitch;
  int64_t pool_bstride;
};

// Grouped launches: one layer of the forwards of several grids (one sample
// each) in one launch. Each grid is a member with its own geometry and
// buffers; `skip` points at the member's solve-decided flag (nonzero: the
// member's workgroups return at once), or is null.
struct ConvMember {
  ConvGeo g;
  const bf16_t* x;
  const bf16_t* eta;
  bf16_t* y;
  float* kpart;         // room for the member's K-split partial sums
  const int32_t* skip;
  int wg0;              // first workgroup of the member along x
  int nwt;              // workgroups per K share (runs of tiles)
  int ks;               // K shares: the split the member's own launch uses
  int kwg0;             // first workgroup of the member in the K-split sum (none without a split)
  int tn;               // the member's own tile width (0: the default), which sets that split
  int pad_;
};
struct PackMember {     // input scaling (sum of squares, then the packed input)
  const float* r;
  int64_t n;
  double* part;
  bf16_t* xin;
  const int32_t* skip;
};
// DeepONet output fused into the epilogue of the last decoder convolution:
// y = gamma * (D0 . fold[p][0:c0] + fold[p][c0]) per pixel p, fold rows of
// `pitch` floats (a per-grid constant), y [samples][pixels] FP32; fold null:
// no fused output.
struct OutFold {
  const float* fold;
  const float* gamma;
  float* y;
  int pitch;
  int c0;
};
struct OutMember {      // DeepONet output
  int64_t npix;
  const bf16_t* d0;
  const float* fold;
  float* y;
  const int32_t* skip;
};

// Number of 32-wide MFMA K-steps of an input-channel chunk of ck channels
// for a kernel with `taps` taps (taps x ck/8 eight-channel groups, rounded up
// to groups of four).
__host__ __device__ __forceinline__ int conv_chunk_steps(int taps, int ck) { return (taps * (ck / 8) + 3) / 4; }

// Length of one output channel's row in the packed BF16 weight layout.
__host__ __device__ __forceinline__ int conv_packed_k(int taps, int cin8) {
  int k = 0;
  for (int c0 = 0; c0 < cin8; c0 += kConvCK) {
    const int ck = (cin8 - c0) < kConvCK ? (cin8 - c0) : kConvCK;
    k += conv_chunk_steps(taps, ck) * 32;
  }
  return k;
}

}  // namespace ppe
