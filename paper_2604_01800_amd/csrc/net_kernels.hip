// Network kernels: Mesh-Conv implicit-GEMM convolutions on BF16 MFMA, the
// grid-derived constants of the DeepONet (local weights eta, trunk basis),
// pooling, input scaling and the DeepONet output (Sec. 2.4, Eqs. 17-18).
#include <algorithm>
#include <type_traits>
#include <vector>

#include "common.hpp"
#include "net_common.hpp"
#include "net_kernels.hpp"

namespace ppe {

// ---------------------------------------------------------------------------
// Convolution as an implicit GEMM: out[px][co] = sum_k Wp[co][k] * Xbar[px, k]
// with k running over (tap, input channel). A workgroup owns TN output
// channels of one sample and a run of consecutive 16 x 16 pixel tiles; wave w
// computes tile rows 4w .. 4w+3, so each K-step issues (TN/16) x 4 MFMA
// 16x16x32 BF16 (A = weights, M = output channels; B = staged inputs, N = 16
// pixels of one tile row; FP32 accumulation) and every operand fragment
// feeds 4 (or TN/16) of them.
//
// The work of a workgroup is a list of items (tile, chunk of 32 input
// channels). For each item the input chunk with its 3x3 halo, multiplied by
// the Mesh-Conv local weight eta on the way (Eq. 18), and the chunk's slice
// of the packed weights are written to LDS (a workgroup with one chunk
// stages its weight slice once); an item's loads are issued before the
// barrier that waits for the other waves' MFMA loops of the item before, and
// the loop itself reads only LDS (fragments one K-step ahead). On tiles whose
// halo lies inside the image every load address is a per-thread offset fixed
// for the launch plus a scalar base. Each lane's eight consecutive K values are one (tap,
// 8-channel group); the packed weight layout enumerates the groups of a chunk
// in the same order, zero-filled to a multiple of four groups. Weight rows
// past cout read as zero through a buffer resource that ends at the last
// output channel. TAPS = 9 (3x3, zero padding) or 1 (1x1). UP = the output is
// written to the 2x nearest-upsampled pixels of a finer level.
constexpr int kCTH = 16, kCTW = 16;  // pixel tile of the convolution kernel

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// Two BF16 values (one word) times one factor each, back to BF16 by one
// packed round-to-nearest-even conversion.
__device__ __forceinline__ uint32_t mul_bf16x2(uint32_t v, float lo, float hi) {
  const float a = __builtin_bit_cast(float, v << 16) * lo;
  const float b = __builtin_bit_cast(float, v & 0xffff0000u) * hi;
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){a, b}, bf16x2_t));
}

// Eight BF16 values times eight BF16 weights (one local weight per input channel).
__device__ __forceinline__ uint4 mul_bf16x8(uint4 v, uint4 e) {
  auto lo = [](uint32_t w) { return __builtin_bit_cast(float, w << 16); };
  auto hi = [](uint32_t w) { return __builtin_bit_cast(float, w & 0xffff0000u); };
  return make_uint4(mul_bf16x2(v.x, lo(e.x), hi(e.x)), mul_bf16x2(v.y, lo(e.y), hi(e.y)),
                    mul_bf16x2(v.z, lo(e.z), hi(e.z)), mul_bf16x2(v.w, lo(e.w), hi(e.w)));
}

// Eight BF16 values times one BF16 weight (one local weight per node).
__device__ __forceinline__ uint4 mul_bf16x8_s(uint4 v, uint32_t e16) {
  const float e = __builtin_bit_cast(float, e16 << 16);
  return make_uint4(mul_bf16x2(v.x, e, e), mul_bf16x2(v.y, e, e), mul_bf16x2(v.z, e, e), mul_bf16x2(v.w, e, e));
}

// Local-weight forms of a convolution: none, one per input channel (a map
// laid out as the input), one per node (a [H][W] map).
enum { kEtaNone = 0, kEtaChannel = 1, kEtaNode = 2 };

template <int TN, int TAPS>
struct ConvShape {
  static constexpr int HALO = TAPS == 9 ? 1 : 0;
  static constexpr int LW = kCTW + 2 * HALO, LH = kCTH + 2 * HALO;
  static constexpr int NPIX = LW * LH;
  // input channels staged per item: 32 for 3x3 layers, 64 for 1x1 layers (the
  // packed weight layout is the same: a full 64-channel chunk of a 1x1 layer
  // is two full 32-channel chunks)
  static constexpr int CK = TAPS == 9 ? kConvCK : 2 * kConvCK;
  static constexpr int G8 = CK / 8;                             // 8-channel groups of a staged pixel
  static constexpr int PPR = 256 / G8;                          // pixels staged per round of 256 threads
  static constexpr int CKP = CK + 8;                            // LDS pitch of a staged pixel (bf16)
  static constexpr int SMAX = (TAPS * G8 + 3) / 4;              // K-steps of a full chunk
  static constexpr int WQ = SMAX * 4;                           // 8-value groups of a full weight row
  static constexpr int WKP = SMAX * 32 + 8;                     // LDS pitch of a staged weight row
  static constexpr int NU = (NPIX + PPR - 1) / PPR;             // staged pixels per thread
  static constexpr int NW = (TN * WQ + 255) / 256;              // weight groups per thread
};

// Registers of one item's loads, between issue and the write to LDS.
template <int TN, int TAPS, int ETA>
struct ConvStage {
  static constexpr int NU = ConvShape<TN, TAPS>::NU;
  uint4 x[NU], w[ConvShape<TN, TAPS>::NW];
  uint4 e[ETA == kEtaChannel ? NU : 1];
  uint32_t e1[ETA == kEtaNode ? NU : 1];
};

// This thread's staged pixels, fixed for the launch: pixel i sits at (ly, lx)
// of the halo tile; xo[i] is its 8-channel group's byte offset from the halo
// tile's first pixel in the input, eo[i] its byte offset in a per-node map
// (both out of range for the slots past the halo tile).
template <int TN, int TAPS>
struct ConvLane {
  static constexpr int NU = ConvShape<TN, TAPS>::NU;
  uint32_t xo[NU], eo[NU];
};

// Kept in registers for the launch where they fit (32 output channels per
// workgroup); recomputed per item (about six VALU operations a pixel) where
// the 64-channel kernel has no registers to spare.
template <int TN>
constexpr bool kKeepLane = TN == 32;

template <int TN, int TAPS>
__device__ __forceinline__ ConvLane<TN, TAPS> conv_lane(const ConvGeo& g) {
  using S = ConvShape<TN, TAPS>;
  ConvLane<TN, TAPS> ln;
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));  // not hoisted out of the item loop where recomputed
  const int c8 = tid % S::G8;
#pragma unroll
  for (int i = 0; i < S::NU; ++i) {
    const int pix = tid / S::G8 + S::PPR * i;
    const int ly = pix / S::LW, lx = pix - ly * S::LW;
    const uint32_t rel = (uint32_t)(ly * g.W + lx);
    const bool ok = pix < S::NPIX;
    ln.xo[i] = ok ? rel * (uint32_t)(g.x_pitch * 2) + (uint32_t)c8 * 16u : 0x80000000u;
    ln.eo[i] = ok ? rel * 2u : 0x80000000u;
  }
  return ln;
}

// Loads of a chunk's weight slice (weight rows past cout read as zero),
// and their write to LDS.
template <int TN, int TAPS>
__device__ __forceinline__ void conv_issue_w(uint4* w, __amdgpu_buffer_rsrc_t wr, int Kp,
                                             int co0, int ck8, int kbase) {
  using S = ConvShape<TN, TAPS>;
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int wq = conv_chunk_steps(TAPS, ck8 * 8) * 4;  // 8-value groups per weight row of this chunk
#pragma unroll
  for (int i = 0; i < S::NW; ++i) {
    const int u = tid + 256 * i;
    const int r = u / S::WQ, q = u - r * S::WQ;
    const bool ok = r < TN && q < wq;
    const uint32_t off = ok ? (uint32_t)(((co0 + r) * Kp + kbase + q * 8) * 2) : 0x80000000u;
    w[i] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(wr, (int)off, 0, 0));
  }
}

template <int TN, int TAPS>
__device__ __forceinline__ void conv_commit_w(const uint4* w, int ck8, bf16_t* s_w) {
  using S = ConvShape<TN, TAPS>;
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int wq = conv_chunk_steps(TAPS, ck8 * 8) * 4;
#pragma unroll
  for (int i = 0; i < S::NW; ++i) {
    const int u = tid + 256 * i;
    const int r = u / S::WQ, q = u - r * S::WQ;
    if (r < TN && q < wq) *(uint4*)(s_w + r * S::WKP + q * 8) = w[i];
  }
}

// Issues the loads of one item: thread t stages the 8-channel group t % G8 of
// the halo pixels t / G8, t / G8 + PPR, ... and a share of the weight slice
// (unless the slice is already in LDS). Inputs are read through buffer
// resources over one sample: input channels below g.cu from the coarse
// source (xur, half the resolution), those below g.c1 from the input buffer
// (xr), the others from the second source (x1r). On a tile whose halo
// lies inside the image and a full chunk of the input buffer, every offset is
// this thread's fixed one plus a scalar base; otherwise halo pixels outside
// the image (and channel groups past the chunk or in the other source) get
// an offset past the end, which reads as zero.
template <int TN, int TAPS, int ETA, bool XU>
__device__ __forceinline__ void conv_issue(ConvStage<TN, TAPS, ETA>& st, const ConvLane<TN, TAPS>& ln,
                                           const ConvGeo& g, __amdgpu_buffer_rsrc_t xr, __amdgpu_buffer_rsrc_t x1r,
                                           __amdgpu_buffer_rsrc_t xur, __amdgpu_buffer_rsrc_t er,
                                           __amdgpu_buffer_rsrc_t wr, int Kp, int co0, int py0, int px0, int c0,
                                           int ck8, int kbase, bool fast, bool fastu, bool wload) {
  using S = ConvShape<TN, TAPS>;
  if (XU && fastu) {
    // a full chunk of the coarse source on an interior tile: halo pixel
    // (ly, lx) reads coarse pixel (py0 / 2 - 1 + (ly + 1) / 2, px0 / 2 - 1 +
    // (lx + 1) / 2) (py0, px0 even), a per-thread offset plus a scalar base
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int c8 = tid % S::G8;
    const int Wc = g.W >> 1;
    const int ubase = ((py0 >> 1) - S::HALO) * Wc + ((px0 >> 1) - S::HALO);
    const int xb = (ubase * g.xu_pitch + c0) * 2;
    const int pbase = (py0 - S::HALO) * g.W + (px0 - S::HALO);
#pragma unroll
    for (int i = 0; i < S::NU; ++i) {
      const int pix = tid / S::G8 + S::PPR * i;
      const int ly = pix / S::LW, lx = pix - ly * S::LW;
      const bool ok = pix < S::NPIX;
      const uint32_t rel = (uint32_t)(((ly + S::HALO) >> 1) * Wc + ((lx + S::HALO) >> 1));
      const uint32_t off = ok ? rel * (uint32_t)(g.xu_pitch * 2) + (uint32_t)c8 * 16u : 0x80000000u;
      st.x[i] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(xur, (int)off, xb, 0));
      if constexpr (ETA == kEtaNode) {
        const uint32_t eo = ok ? (uint32_t)(ly * g.W + lx) * 2u : 0x80000000u;
        st.e1[i] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(er, (int)eo, pbase * 2, 0);
      }
      if constexpr (ETA == kEtaChannel) {  // the map is laid out with pitch cin8
        const uint32_t eo = ok ? (uint32_t)(ly * g.W + lx) * (uint32_t)(g.cin8 * 2) + (uint32_t)(c0 + c8 * 8) * 2u
                               : 0x80000000u;
        st.e[i] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(er, (int)eo, pbase * g.cin8 * 2, 0));
      }
    }
  } else if (fast) {
    const ConvLane<TN, TAPS> lf = kKeepLane<TN> ? ln : conv_lane<TN, TAPS>(g);
    const int pbase = (py0 - S::HALO) * g.W + (px0 - S::HALO);  // first halo pixel (>= 0 here)
    const int xb = (pbase * g.x_pitch + c0) * 2;
#pragma unroll
    for (int i = 0; i < S::NU; ++i) {
      st.x[i] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(xr, (int)lf.xo[i], xb, 0));
      if constexpr (ETA == kEtaChannel)  // (the fast path runs only when the map's pitch is the input's)
        st.e[i] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(er, (int)lf.xo[i], xb, 0));
      if constexpr (ETA == kEtaNode)
        st.e1[i] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(er, (int)lf.eo[i], pbase * 2, 0);
    }
  } else {
    // recomputed per item (cheap next to the fast path's share) rather than kept live
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int c8 = tid % S::G8;
    const int cg = c0 + c8 * 8;  // this thread's first input channel
    const bool cg_ok = c8 < ck8;
    const bool srcu = XU && cg < g.cu, src1 = cg >= g.c1;
    // sources the chunk touches (uniform)
    const bool anyu = XU && c0 < g.cu, any0 = c0 < g.c1 && (!XU || c0 + ck8 * 8 > g.cu), any1 = c0 + ck8 * 8 > g.c1;
#pragma unroll
    for (int i = 0; i < S::NU; ++i) {
      const int pix = tid / S::G8 + S::PPR * i;
      const int ly = pix / S::LW, lx = pix - ly * S::LW;
      const int gy = py0 + ly - S::HALO, gx = px0 + lx - S::HALO;
      const bool in = cg_ok && pix < S::NPIX && gy >= 0 && gy < g.H && gx >= 0 && gx < g.W;
      const uint32_t pi = (uint32_t)(gy * g.W + gx);
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (anyu) {
        const uint32_t pu = (uint32_t)((gy >> 1) * (g.W >> 1) + (gx >> 1));
        const uint32_t off = in && srcu ? pu * (uint32_t)(g.xu_pitch * 2) + (uint32_t)cg * 2u : 0x80000000u;
        v = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(xur, (int)off, 0, 0));
      }
      if (any0) {
        const uint32_t off =
            in && !src1 && !srcu ? pi * (uint32_t)(g.x_pitch * 2) + (uint32_t)cg * 2u : 0x80000000u;
        const uint4 w = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(xr, (int)off, 0, 0));
        v = make_uint4(v.x | w.x, v.y | w.y, v.z | w.z, v.w | w.w);
      }
      if (any1) {
        const uint32_t off =
            in && src1 ? pi * (uint32_t)(g.x1_pitch * 2) + (uint32_t)(cg - g.c1) * 2u : 0x80000000u;
        const uint4 w = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(x1r, (int)off, 0, 0));
        v = make_uint4(v.x | w.x, v.y | w.y, v.z | w.z, v.w | w.w);
      }
      st.x[i] = v;
      if constexpr (ETA == kEtaChannel) {  // the map is laid out with pitch cin8
        const uint32_t eo = in ? pi * (uint32_t)(g.cin8 * 2) + (uint32_t)cg * 2u : 0x80000000u;
        st.e[i] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(er, (int)eo, 0, 0));
      }
      if constexpr (ETA == kEtaNode) {
        const uint32_t eo = in ? pi * 2u : 0x80000000u;
        st.e1[i] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(er, (int)eo, 0, 0);
      }
    }
  }
  if (wload) conv_issue_w<TN, TAPS>(st.w, wr, Kp, co0, ck8, kbase);
}

// Writes one item's staged registers to LDS (inputs times eta).
template <int TN, int TAPS, int ETA>
__device__ __forceinline__ void conv_commit(const ConvStage<TN, TAPS, ETA>& st, int ck8, bool wload, bf16_t* s_x,
                                            bf16_t* s_w) {
  using S = ConvShape<TN, TAPS>;
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int c8 = tid % S::G8;
  if (c8 < ck8) {
#pragma unroll
    for (int i = 0; i < S::NU; ++i) {
      const int pix = tid / S::G8 + S::PPR * i;
      if (pix < S::NPIX) {
        uint4 v = st.x[i];
        if constexpr (ETA == kEtaChannel) v = mul_bf16x8(v, st.e[i]);
        if constexpr (ETA == kEtaNode) v = mul_bf16x8_s(v, st.e1[i]);
        *(uint4*)(s_x + pix * S::CKP + c8 * 8) = v;
      }
    }
  }
  if (wload) conv_commit_w<TN, TAPS>(st.w, ck8, s_w);
}

// MFMA loop over the K-steps of one staged item. B fragments (staged
// inputs) are read one step ahead, A fragments (staged weights) just before
// use.
template <int TN, int TAPS, int CK8>
__device__ __forceinline__ void conv_mfma(f32x4_t (&acc)[TN / 16][4], const bf16_t* s_x, const bf16_t* s_w,
                                          int ck8_rt, int lane, int wv) {
  using S = ConvShape<TN, TAPS>;
  constexpr int MT = TN / 16, NT = 4;
  const int ck8 = CK8 ? CK8 : ck8_rt;
  const int steps = conv_chunk_steps(TAPS, ck8 * 8);
  auto bfrags = [&](int st, bf16x8_t* bf) {
    const int G = st * 4 + (lane >> 4);
    int tap = G / ck8;
    const int c8 = G - tap * ck8;
    if (tap >= TAPS) tap = TAPS - 1;  // zero-weight padding group: any in-bounds input
    const int dy = TAPS == 9 ? tap / 3 : 0, dx = TAPS == 9 ? tap % 3 : 0;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int pix = (NT * wv + nt + dy) * S::LW + (lane & 15) + dx;
      bf[nt] = *(const bf16x8_t*)(s_x + pix * S::CKP + c8 * 8);
    }
  };
  const bf16_t* wrow = s_w + (lane & 15) * S::WKP + (lane >> 4) * 8;
  bf16x8_t bfr[NT];
  bfrags(0, bfr);
  for (int st = 0; st < steps; ++st) {
    bf16x8_t afr[MT], bnx[NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) afr[mt] = *(const bf16x8_t*)(wrow + mt * 16 * S::WKP + st * 32);
    if (st + 1 < steps) bfrags(st + 1, bnx);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[mt], bfr[nt], acc[mt][nt], 0, 0, 0);
    if (st + 1 < steps) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) bfr[nt] = bnx[nt];
    }
  }
}

// WSTAT: the workgroup has one input-channel chunk, so its weight slice is
// staged once, before its first tile.
//
// GRP: a grouped launch over the forwards of several grids. The geometry,
// buffers and K split of each grid come from the member table `mem` (nmem
// entries ordered by their first workgroup along x); a workgroup finds its
// member, returns at once when the member's solve has decided, and then does
// exactly the work of the same tile run in the member's own launch.
// One 4-channel group of the DeepONet output contraction: BF16 activations
// d (two packed pairs) times fold weights w, a product and three FMAs in
// channel order. Both output paths (the separate kernel and the fused
// convolution epilogue) use it, so they round alike.
__device__ __forceinline__ float out_group4(uint2 d, float4 w) {
  float e = __fmul_rn(bf2f((bf16_t)(d.x & 0xffff)), w.x);
  e = __fmaf_rn(bf2f((bf16_t)(d.x >> 16)), w.y, e);
  e = __fmaf_rn(bf2f((bf16_t)(d.y & 0xffff)), w.z, e);
  return __fmaf_rn(bf2f((bf16_t)(d.y >> 16)), w.w, e);
}

template <int TN, int TAPS, bool UP, int ETA, bool WSTAT, bool GRP, bool XU, bool OUTF = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_conv(
    ConvGeo g, const bf16_t* __restrict__ x, const bf16_t* __restrict__ eta, const bf16_t* __restrict__ wp, int Kp,
    const float* __restrict__ bias, bf16_t* __restrict__ y, int tiles_per_wg, float* __restrict__ kpart, int ksplit,
    const ConvMember* __restrict__ mem, int nmem, OutFold of) {
  using S = ConvShape<TN, TAPS>;
  constexpr int MT = TN / 16, NT = 4;
  __shared__ __attribute__((aligned(16))) bf16_t s_x[S::NPIX * S::CKP];
  __shared__ __attribute__((aligned(16))) bf16_t s_w[TN * S::WKP];
  __shared__ __attribute__((aligned(16))) float s_b[TN];

  int t0, smp, ksp, nbs;  // first tile, sample, K share, samples of the launch
  if constexpr (GRP) {
    int lo = 0, hi = nmem - 1;  // the last member whose first workgroup is <= blockIdx.x
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (mem[mid].wg0 <= (int)blockIdx.x) lo = mid;
      else hi = mid - 1;
    }
    const ConvMember& M = mem[lo];
    // a uniform branch (the flag's value taken from the first lane), so that
    // the member's fields stay in scalar registers
    if (M.skip && __builtin_amdgcn_readfirstlane(*M.skip) != 0) return;
    g = M.g;
    x = M.x;
    eta = M.eta;
    y = M.y;
    kpart = M.kpart;
    ksplit = M.ks;
    const int local = (int)blockIdx.x - M.wg0;
    ksp = local / M.nwt;
    t0 = (local - ksp * M.nwt) * tiles_per_wg;
    smp = 0;
    nbs = 1;
  } else {
    t0 = blockIdx.x * tiles_per_wg;
    smp = blockIdx.z / ksplit;
    ksp = blockIdx.z - smp * ksplit;
    nbs = gridDim.z / ksplit;
  }
  const int tiles_x = (g.W + kCTW - 1) / kCTW;
  const int tiles = tiles_x * ((g.H + kCTH - 1) / kCTH);
  const int nt_wg = min(tiles_per_wg, tiles - t0);
  const int co0 = blockIdx.y * TN;
  x += smp * g.x_bstride;
  y += smp * g.y_bstride;
  if (ETA != kEtaNone) eta += smp * g.e_bstride;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // the output channels' biases (0 past cout), read by the epilogue after
  // the first item's barriers
  if (threadIdx.x < TN) s_b[threadIdx.x] = (bias && co0 + (int)threadIdx.x < g.cout) ? bias[co0 + threadIdx.x] : 0.f;
  const __amdgpu_buffer_rsrc_t wr =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<bf16_t*>(wp), (short)0, (int)((int64_t)g.cout * Kp * 2), 0x00020000);
  const int in_bytes = (int)((int64_t)g.H * g.W * g.x_pitch * 2);  // one sample of the input
  const __amdgpu_buffer_rsrc_t xr =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<bf16_t*>(x), (short)0, in_bytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t x1r = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<bf16_t*>(g.x1 ? g.x1 + smp * g.x1_bstride : x), (short)0,
      g.x1 ? (int)((int64_t)g.H * g.W * g.x1_pitch * 2) : 0, 0x00020000);
  const __amdgpu_buffer_rsrc_t xur = XU ? __builtin_amdgcn_make_buffer_rsrc(
                                               const_cast<bf16_t*>(g.xu + smp * g.xu_bstride), (short)0,
                                               (int)((int64_t)(g.H / 2) * (g.W / 2) * g.xu_pitch * 2), 0x00020000)
                                         : xr;
  const int eta_bytes = (int)((int64_t)g.H * g.W * (ETA == kEtaNode ? 1 : g.cin8) * 2);
  const __amdgpu_buffer_rsrc_t er = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<bf16_t*>(ETA != kEtaNone ? eta : x), (short)0, eta_bytes, 0x00020000);
  const int HO = UP ? 2 * g.H : g.H, WO = UP ? 2 * g.W : g.W;
  const __amdgpu_buffer_rsrc_t yr =
      __builtin_amdgcn_make_buffer_rsrc(y, (short)0, (int)((int64_t)HO * WO * g.y_pitch * 2), 0x00020000);
  // the 2 x 2 pooled output into the next level, when asked for
  const bool pool = g.pool_y != nullptr;
  const __amdgpu_buffer_rsrc_t pr = __builtin_amdgcn_make_buffer_rsrc(
      pool ? g.pool_y + smp * g.pool_bstride : y, (short)0,
      pool ? (int)((int64_t)(g.H / 2) * (g.W / 2) * g.pool_pitch * 2) : 0, 0x00020000);
  ConvLane<TN, TAPS> ln;
  if constexpr (kKeepLane<TN>) ln = conv_lane<TN, TAPS>(g);
  // input-channel chunks of this workgroup: all of them, or its share when
  // the K loop is split over ksplit workgroups
  const int nch_all = (g.cin8 + S::CK - 1) / S::CK;
  const int cps = (nch_all + ksplit - 1) / ksplit;
  const int c_lo = ksp * cps;
  const int nch = min(cps, nch_all - c_lo);
  const int items = nt_wg * nch;

  f32x4_t acc[MT][NT];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[m][n] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  if constexpr (WSTAT) {
    // the one chunk's weight slice, before the first item (whose barriers
    // order it before the first MFMA loop)
    const int ck8 = min(S::CK, g.cin8 - c_lo * S::CK) / 8;
    uint4 w[S::NW];
    conv_issue_w<TN, TAPS>(w, wr, Kp, co0, ck8, c_lo * S::SMAX * 32);
    conv_commit_w<TN, TAPS>(w, ck8, s_w);
  }
  constexpr bool wload = !WSTAT;
  // the loads of item it
  auto issue = [&](ConvStage<TN, TAPS, ETA>& st, int it) {
    const int t = t0 + it / nch, c = c_lo + it - (it / nch) * nch;
    const int c0 = c * S::CK;
    const int ck8 = min(S::CK, g.cin8 - c0) / 8;
    const int py0 = (t / tiles_x) * kCTH, px0 = (t % tiles_x) * kCTW;
    const bool interior =
        py0 >= S::HALO && px0 >= S::HALO && py0 + kCTH + S::HALO <= g.H && px0 + kCTW + S::HALO <= g.W;
    const bool fast = ck8 == S::G8 && (!XU || c0 >= g.cu) && c0 + S::CK <= g.c1 &&
                      (ETA != kEtaChannel || g.x_pitch == g.cin8) && interior;
    const bool fastu = XU && ck8 == S::G8 && c0 + S::CK <= g.cu && interior;
    conv_issue<TN, TAPS, ETA, XU>(st, ln, g, xr, x1r, xur, er, wr, Kp, co0, py0, px0, c0, ck8, c * S::SMAX * 32, fast,
                              fastu, wload);
  };
  for (int it = 0; it < items; ++it) {
    const int t = t0 + it / nch, c = c_lo + it - (it / nch) * nch;
    const int ck8 = min(S::CK, g.cin8 - c * S::CK) / 8;
    const int py0 = (t / tiles_x) * kCTH, px0 = (t % tiles_x) * kCTW;
    // in flight while the other waves finish the previous item (declared here:
    // nothing of it is live from one item to the next). Issuing the next
    // item's loads before the current MFMA loop instead costs the 32-channel
    // kernel a resident workgroup per CU and was slower.
    ConvStage<TN, TAPS, ETA> stg;
    issue(stg, it);
    __syncthreads();  // the previous item's MFMA loop is done with LDS
    conv_commit<TN, TAPS, ETA>(stg, ck8, wload, s_x, s_w);
    __syncthreads();

    if (ck8 == S::G8)
      conv_mfma<TN, TAPS, S::G8>(acc, s_x, s_w, ck8, lane, wv);
    else
      conv_mfma<TN, TAPS, 0>(acc, s_x, s_w, ck8, lane, wv);
    if (c + 1 < c_lo + nch) continue;

    // Epilogue of tile t: lane holds out[co0 + mt*16 + 4*(lane>>4) + j][pixel (row NT*w+nt, col lane&15)].
    if (ksplit > 1) {
      // partial sums of this share of K, [ksplit][sample][pixel][gridDim.y * TN] FP32
      const int cp = gridDim.y * TN;
      float* pp = kpart + ((int64_t)ksp * nbs + smp) * g.H * g.W * cp;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int co = co0 + mt * 16 + 4 * (lane >> 4);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int py = py0 + NT * wv + nt, px = px0 + (lane & 15);
          if (co < g.cout && py < g.H && px < g.W)
            *(f32x4_t*)(pp + ((int64_t)py * g.W + px) * cp + co) = acc[mt][nt];
          acc[mt][nt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        }
      }
      continue;
    }
    if constexpr (OUTF) {
      // DeepONet output instead of the stored activations (TN = 32 and
      // c0 <= 32: the workgroup holds every channel of its pixels). The
      // lane's channel group q = 4 mt + (lane >> 4) takes the place of lane q
      // of k_deeponet_out: the same BF16-rounded values, the same group sum,
      // and the same pairwise order across groups (q ^ 4 within the lane, then
      // lanes ^ 32 and ^ 16), so the result is that kernel's bit for bit.
      static_assert(TN == 32 && !UP && !GRP, "fused output: 32 output channels per workgroup, plain launch");
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int py = py0 + NT * wv + nt, px = px0 + (lane & 15);
        const bool pok = py < g.H && px < g.W;
        const int64_t pix = (int64_t)py * g.W + px;
        float sq[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int col = mt * 16 + 4 * (lane >> 4);
          const f32x4_t b = *(const f32x4_t*)(s_b + col);
          float v[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) v[j] = acc[mt][nt][j] + b[j];
          if (g.act == 1) {
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = __builtin_amdgcn_fmed3f(v[j], 0.f, __builtin_inff());
          } else if (g.act == 2) {
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = tanh_nn(v[j]);
          }
          const uint2 pk = {__builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){v[0], v[1]}, bf16x2_t)),
                            __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){v[2], v[3]}, bf16x2_t))};
          sq[mt] = 0.f;
          if (pok && col < of.c0) sq[mt] += out_group4(pk, *(const float4*)(of.fold + pix * of.pitch + col));
          acc[mt][nt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        }
        float sv = sq[0] + sq[1];
        sv += __shfl_xor(sv, 32);
        sv += __shfl_xor(sv, 16);
        if (pok && lane < 16)
          of.y[(int64_t)smp * g.H * g.W + pix] = of.gamma[0] * (sv + of.fold[pix * of.pitch + of.c0]);
      }
      continue;
    }
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int col = mt * 16 + 4 * (lane >> 4);  // first of this lane's 4 channels within the workgroup's TN
      const int co = co0 + col;
      const bool cok = co < g.cout;
      const f32x4_t b = *(const f32x4_t*)(s_b + col);
      u32x2 pk[NT];  // the stored BF16 values (pooling reads them back)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int py = py0 + NT * wv + nt, px = px0 + (lane & 15);
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = acc[mt][nt][j] + b[j];
        if (g.act == 1) {
#pragma unroll
          for (int j = 0; j < 4; ++j) v[j] = __builtin_amdgcn_fmed3f(v[j], 0.f, __builtin_inff());
        } else if (g.act == 2) {
#pragma unroll
          for (int j = 0; j < 4; ++j) v[j] = tanh_nn(v[j]);
        }
        const u32x2 packed = {__builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){v[0], v[1]}, bf16x2_t)),
                              __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){v[2], v[3]}, bf16x2_t))};
        pk[nt] = packed;
        if (!cok || py >= g.H || px >= g.W) continue;
        if (!UP) {
          const uint32_t o = (uint32_t)(((py * WO + px) * g.y_pitch + g.y_off + co) * 2);
          __builtin_amdgcn_raw_buffer_store_b64(packed, yr, (int)o, 0, 0);
        } else {
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int bb = 0; bb < 2; ++bb) {
              const uint32_t o = (uint32_t)((((2 * py + a) * WO + 2 * px + bb) * g.y_pitch + g.y_off + co) * 2);
              __builtin_amdgcn_raw_buffer_store_b64(packed, yr, (int)o, 0, 0);
            }
        }
      }
      if (!UP && pool) {
        // 2 x 2 average into the next level: rows nt, nt + 1 of this lane and
        // the same rows of the next column's lane; the sum in the order and
        // rounding of the pooling kernel, from the stored BF16 values
#pragma unroll
        for (int nt = 0; nt < NT; nt += 2) {
          const uint32_t w[4][2] = {{pk[nt].x, pk[nt].y},
                                    {(uint32_t)__shfl_xor((int)pk[nt].x, 1), (uint32_t)__shfl_xor((int)pk[nt].y, 1)},
                                    {pk[nt + 1].x, pk[nt + 1].y},
                                    {(uint32_t)__shfl_xor((int)pk[nt + 1].x, 1),
                                     (uint32_t)__shfl_xor((int)pk[nt + 1].y, 1)}};
          float sm[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              sm[2 * h] += bf2f((bf16_t)(w[q][h] & 0xffff));
              sm[2 * h + 1] += bf2f((bf16_t)(w[q][h] >> 16));
            }
          const int py = py0 + NT * wv + nt, px = px0 + (lane & 15);
          if (cok && (lane & 1) == 0 && py < g.H && px < g.W) {
            const u32x2 pooled = {(uint32_t)f2bf(0.25f * sm[0]) | ((uint32_t)f2bf(0.25f * sm[1]) << 16),
                                  (uint32_t)f2bf(0.25f * sm[2]) | ((uint32_t)f2bf(0.25f * sm[3]) << 16)};
            const uint32_t o = (uint32_t)((((py >> 1) * (g.W >> 1) + (px >> 1)) * g.pool_pitch + co) * 2);
            __builtin_amdgcn_raw_buffer_store_b64(pooled, pr, (int)o, 0, 0);
          }
        }
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    }
  }
}

// Sum of the K-split partials of a convolution, in a fixed order, then bias,
// activation and the BF16 store of the unsplit epilogue (UP: to the 2 x 2
// finer pixels). One thread per (pixel, 4 output channels); cp = channel pitch
// of the partials.
// GRP: a grouped launch; the workgroups of the members with a split follow
// one another (member table `mem` of nb entries, ordered by kwg0), and those
// of a member whose solve has decided return.
template <bool UP, bool GRP>
__global__ __launch_bounds__(256) void k_conv_ksum(ConvGeo g, int nb, int ksplit, int cp,
                                                   const float* __restrict__ kpart, const float* __restrict__ bias,
                                                   bf16_t* __restrict__ y, const ConvMember* __restrict__ mem) {
  int smp = blockIdx.y;
  int64_t blk = blockIdx.x;
  if constexpr (GRP) {
    int lo = 0, hi = nb - 1;  // the last member whose first workgroup is <= blockIdx.x
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (mem[mid].kwg0 <= (int)blockIdx.x) lo = mid;
      else hi = mid - 1;
    }
    const ConvMember& M = mem[lo];
    if (M.ks < 2 || (M.skip && __builtin_amdgcn_readfirstlane(*M.skip) != 0)) return;
    g = M.g;
    nb = 1;
    ksplit = M.ks;
    kpart = M.kpart;
    y = M.y;
    smp = 0;
    blk -= M.kwg0;
  }
  // one thread per 4 output channels of a pixel; with the pooled output the
  // four pixels of a 2 x 2 block are the four lanes of a quad
  const bool pool = !UP && g.pool_y != nullptr;
  const int q4 = g.cout / 4;
  const int64_t hw = (int64_t)g.H * g.W;
  const int64_t i = blk * 256 + threadIdx.x;
  if (i >= hw * q4) return;  // whole quads: hw * q4 is a multiple of 4 with pooling
  int64_t p;
  int co, sub = 0;
  if (!pool) {
    p = i / q4;
    co = (int)(i - p * q4) * 4;
  } else {
    const int64_t t = i >> 2;  // (pooled pixel, channel quad)
    sub = (int)(i & 3);        // (row, column) of the pixel in its block
    const int64_t u = t / q4;
    co = (int)(t - u * q4) * 4;
    const int Wo = g.W / 2;
    const int yo = (int)(u / Wo), xo = (int)(u - (int64_t)yo * Wo);
    p = (int64_t)(2 * yo + (sub >> 1)) * g.W + 2 * xo + (sub & 1);
  }
  const int64_t kstride = (int64_t)nb * hw * cp;
  const float* src = kpart + ((int64_t)smp * hw + p) * cp + co;
  f32x4_t a = *(const f32x4_t*)src;
  for (int k = 1; k < ksplit; ++k) {
    const f32x4_t b = *(const f32x4_t*)(src + k * kstride);
    a[0] += b[0];
    a[1] += b[1];
    a[2] += b[2];
    a[3] += b[3];
  }
  float v[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float t = a[j] + (bias ? bias[co + j] : 0.f);
    if (g.act == 1) t = fmaxf(t, 0.f);
    else if (g.act == 2) t = tanh_nn(t);
    v[j] = t;
  }
  const uint2 packed = make_uint2((uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16),
                                  (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16));
  y += smp * g.y_bstride;
  const int py = (int)(p / g.W), px = (int)(p - (int64_t)py * g.W);
  if (!UP) {
    *(uint2*)(y + p * g.y_pitch + g.y_off + co) = packed;
  } else {
    const int W2 = 2 * g.W;
#pragma unroll
    for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
      for (int b2 = 0; b2 < 2; ++b2)
        *(uint2*)(y + ((size_t)(2 * py + a2) * W2 + 2 * px + b2) * g.y_pitch + g.y_off + co) = packed;
  }
  if (pool) {
    // the block's average in the pooling kernel's order (pixels 0..3 of the
    // quad: row-major in the block), from the stored BF16 values
    float sm[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t wx = (uint32_t)__shfl((int)packed.x, q, 4);
      const uint32_t wy = (uint32_t)__shfl((int)packed.y, q, 4);
      sm[0] += bf2f((bf16_t)(wx & 0xffff));
      sm[1] += bf2f((bf16_t)(wx >> 16));
      sm[2] += bf2f((bf16_t)(wy & 0xffff));
      sm[3] += bf2f((bf16_t)(wy >> 16));
    }
    if (sub == 0)
      *(uint2*)(g.pool_y + smp * g.pool_bstride + ((int64_t)(py >> 1) * (g.W >> 1) + (px >> 1)) * g.pool_pitch + co) =
          make_uint2((uint32_t)f2bf(0.25f * sm[0]) | ((uint32_t)f2bf(0.25f * sm[1]) << 16),
                     (uint32_t)f2bf(0.25f * sm[2]) | ((uint32_t)f2bf(0.25f * sm[3]) << 16));
  }
}

// A 1x1 layer of at most 128 output and 128 input channels as a skinny GEMM,
// y[p][co] = act(bias[co] + sum_k W[co][k] x[p][k]). The workgroup stages the
// layer's packed weights in LDS once (A fragments: M = output channels, K =
// input channels); each wavefront then streams 16-pixel tiles, loading the B
// fragments (8 consecutive input channels of one pixel per lane) straight
// from memory two tiles ahead, and computes all output channels of a tile.
// Every input byte is read once. MT = output-channel tiles of 16 (cout <=
// 16 MT); K-steps = Kp / 32 <= 4. GRP: a grouped launch, blockIdx.y the
// member (its geometry and buffers from the member table).
constexpr int kC1KS = 4;                  // K-steps at most (Kp <= 128)
constexpr int kC1WP = kC1KS * 32 + 8;     // LDS pitch of a weight row (bf16)
template <int MT, bool GRP>
__global__ __launch_bounds__(256) void k_conv1x1(ConvGeo g, const bf16_t* __restrict__ x,
                                                 const bf16_t* __restrict__ wp, int Kp,
                                                 const float* __restrict__ bias, bf16_t* __restrict__ y,
                                                 const ConvMember* __restrict__ mem) {
  __shared__ __attribute__((aligned(16))) bf16_t s_w[MT * 16 * kC1WP];
  constexpr int OP = MT * 16 + 8;  // LDS pitch (bf16) of a staged output pixel
  __shared__ __attribute__((aligned(16))) bf16_t s_o[4][16 * OP];  // per wavefront
  const int nks = Kp / 32;
  const int lane = threadIdx.x & 63;
  int smp = blockIdx.y;
  if constexpr (GRP) {
    const ConvMember& M = mem[blockIdx.y];
    if (M.skip && __builtin_amdgcn_readfirstlane(*M.skip) != 0) return;
    g = M.g;
    x = M.x;
    y = M.y;
    smp = 0;
  }
  x += smp * g.x_bstride;
  y += smp * g.y_bstride;
  const int npix = g.H * g.W;
  // weights: rows past cout read as zero
  const __amdgpu_buffer_rsrc_t wr =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<bf16_t*>(wp), (short)0, (int)((int64_t)g.cout * Kp * 2), 0x00020000);
  for (int u = threadIdx.x; u < MT * 16 * (Kp / 8); u += 256) {
    const int r = u / (Kp / 8), q = u - r * (Kp / 8);
    *(uint4*)(s_w + r * kC1WP + q * 8) =
        __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(wr, (int)((r * Kp + q * 8) * 2), 0, 0));
  }
  __syncthreads();
  const __amdgpu_buffer_rsrc_t xr =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<bf16_t*>(x), (short)0, (int)((int64_t)npix * g.x_pitch * 2), 0x00020000);
  const int tiles = (npix + 15) / 16;
  const int wv = blockIdx.x * 4 + (threadIdx.x >> 6), nwv = gridDim.x * 4;
  // B fragments of tile t: channels ks*32 + (lane>>4)*8 of pixel 16t + (lane&15)
  auto bload = [&](int t, bf16x8_t* bf) {
    const int px = t * 16 + (lane & 15);
#pragma unroll
    for (int ks = 0; ks < kC1KS; ++ks) {
      const int k = ks * 32 + (lane >> 4) * 8;
      const uint32_t o = (ks < nks && px < npix && k < g.cin8) ? (uint32_t)(px * g.x_pitch + k) * 2u : 0x80000000u;
      bf[ks] = __builtin_bit_cast(bf16x8_t, __builtin_amdgcn_raw_buffer_load_b128(xr, (int)o, 0, 0));
    }
  };
  const bf16_t* arow = s_w + (lane & 15) * kC1WP + (lane >> 4) * 8;
  float bv[MT][4];  // this lane's output channels' biases
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int co = mt * 16 + 4 * (lane >> 4) + j;
      bv[mt][j] = (bias && co < g.cout) ? bias[co] : 0.f;
    }
  auto tile = [&](int t, const bf16x8_t* bf) {
    f32x4_t acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kC1KS; ++ks) {
      if (ks >= nks) break;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const bf16x8_t af = *(const bf16x8_t*)(arow + mt * 16 * kC1WP + ks * 32);
        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf[ks], acc[mt], 0, 0, 0);
      }
    }
    // the tile's outputs through the wavefront's LDS rows, then stored as
    // 16-byte pieces that cover whole pixel rows
    bf16_t* so = s_o[threadIdx.x >> 6];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int co = mt * 16 + 4 * (lane >> 4);
      float v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v[j] = acc[mt][j] + bv[mt][j];
        if (g.act == 1) v[j] = fmaxf(v[j], 0.f);
        else if (g.act == 2) v[j] = tanh_nn(v[j]);
      }
      *(uint2*)(so + (lane & 15) * OP + co) = make_uint2((uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16),
                                                         (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16));
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int c8n = g.cout / 8;  // 8-channel groups per pixel
#pragma unroll
    for (int e0 = 0; e0 < 16 * MT * 2; e0 += 64) {
      const int e = e0 + lane, q = e / (MT * 2), c8 = e - q * (MT * 2);
      const int px = t * 16 + q;
      if (c8 < c8n && px < npix)
        *(uint4*)(y + (size_t)px * g.y_pitch + g.y_off + c8 * 8) = *(const uint4*)(so + q * OP + c8 * 8);
    }
    __builtin_amdgcn_wave_barrier();
  };
  // two tiles in flight: the loads of tile t + 2 nwv are issued as soon as
  // tile t's fragments are consumed
  bf16x8_t b0[kC1KS], b1[kC1KS];
  int t = wv;
  if (t < tiles) bload(t, b0);
  if (t + nwv < tiles) bload(t + nwv, b1);
  while (t < tiles) {
    tile(t, b0);
    if (t + 2 * nwv < tiles) bload(t + 2 * nwv, b0);
    t += nwv;
    if (t >= tiles) break;
    tile(t, b1);
    if (t + 2 * nwv < tiles) bload(t + 2 * nwv, b1);
    t += nwv;
  }
}

// Packed BF16 weights from the FP32 master layout W[cout_fwd][cin_fwd][taps].
// mode 0: the forward operator (rows = output channels, K over input channels).
// mode 1: the input-gradient operator, a 3x3 (or 1x1) convolution from the
// output-channel space back to the input-channel space with the kernel
// flipped: rows = input channels, K over output channels, tap -> taps-1-tap.
// rows x Kp values; kin8 = K-side channel count padded to 8.
__global__ void k_pack_weights(const float* __restrict__ w, int rows, int kin8, int taps, int Kp, int mode,
                               int cout_fwd, int cin_fwd, bf16_t* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)rows * Kp) return;
  const int row = (int)(idx / Kp);
  int k = (int)(idx - (int64_t)row * Kp);
  float v = 0.f;
  for (int c0 = 0; c0 < kin8; c0 += kConvCK) {
    const int ck = min(kConvCK, kin8 - c0), ck8 = ck / 8;
    const int kw = conv_chunk_steps(taps, ck) * 32;
    if (k < kw) {
      const int G = k / 8, e = k - G * 8;
      if (G < taps * ck8) {
        const int tap = G / ck8, c8 = G - tap * ck8;
        const int ch = c0 + c8 * 8 + e;
        if (mode == 0) {
          if (row < cout_fwd && ch < cin_fwd) v = w[((size_t)row * cin_fwd + ch) * taps + tap];
        } else {
          if (row < cin_fwd && ch < cout_fwd) v = w[((size_t)ch * cin_fwd + row) * taps + (taps - 1 - tap)];
        }
      }
      break;
    }
    k -= kw;
  }
  out[idx] = f2bf(v);
}

// ---------------------------------------------------------------------------
// Mesh-Conv local weight (Eq. 17) of one layer at every pixel of its level:
// eta[p][c] = exp(-Phi(Delta_p)_c^2), Phi = W2 tanh(W1 Delta + b1) + b2, with
// Delta_p = (left, right, down, up) neighbour distances (1D arrays per level).
// Channels c >= cin (padding) get 0.
__global__ void k_eta(int H, int W, int cin, int cin8, int hid, const float* __restrict__ dxl,
                      const float* __restrict__ dxr, const float* __restrict__ dyd, const float* __restrict__ dyu,
                      const float* __restrict__ W1, const float* __restrict__ b1, const float* __restrict__ W2,
                      const float* __restrict__ b2, bf16_t* __restrict__ eta) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)H * W) return;
  const int j = (int)(p / W), i = (int)(p - (int64_t)j * W);
  const float d[4] = {dxl[i], dxr[i], dyd[j], dyu[j]};
  float h[32];
  for (int a = 0; a < hid; ++a) {
    float s = b1[a];
    for (int q = 0; q < 4; ++q) s += W1[a * 4 + q] * d[q];
    h[a] = tanh_nn(s);
  }
  bf16_t* out = eta + p * cin8;
  for (int c = 0; c < cin8; ++c) {
    float e = 0.f;
    if (c < cin) {
      float phi = b2[c];
      for (int a = 0; a < hid; ++a) phi += W2[c * hid + a] * h[a];
      e = exp_nn(-phi * phi);
    }
    out[c] = f2bf(e);
  }
}

// Trunk basis with the branch head folded in. For each pixel: T = trunk(xy)
// (tanh hidden layers, linear output, FP32), then
//   out[p][c] = sum_k Wh[k][c] T_k  (c < C0),   out[p][C0] = sum_k bh[k] T_k,
// so the DeepONet output sum_k (Wh D + bh)_k T_k = D . out[p][0:C0] + out[p][C0].
// A workgroup of 256 threads handles 32 pixels; thread t computes neuron
// t % 128 for pixels 16 * (t / 128) ... +16.
constexpr int kTrunkPix = 32;
__global__ __launch_bounds__(256) void k_trunk_fold(int H, int W, const float* __restrict__ xin,
                                                    const float* __restrict__ yin, const float* __restrict__ params,
                                                    TrunkDesc td, float* __restrict__ out) {
  __shared__ float act[kTrunkPix][129];
  __shared__ float nxt[kTrunkPix][129];
  const int64_t p0 = (int64_t)blockIdx.x * kTrunkPix;
  const int64_t npix = (int64_t)H * W;
  const int t = threadIdx.x, j = t & 127, pg = t >> 7;
  if (t < kTrunkPix) {
    const int64_t p = p0 + t;
    const int64_t pc = p < npix ? p : npix - 1;
    const int jj = (int)(pc / W), ii = (int)(pc - (int64_t)jj * W);
    act[t][0] = xin[ii];
    act[t][1] = yin[jj];
  }
  __syncthreads();
  int nin = 2;
  for (int layer = 0; layer <= td.hidden; ++layer) {
    const bool last = layer == td.hidden;
    const float* Wl = params + td.oW[layer];
    const float* bl = params + td.ob[layer];
    const int nout = last ? td.basis : td.width;
    if (j < nout) {
      float accv[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) accv[q] = bl[j];
      for (int k = 0; k < nin; ++k) {
        const float w = Wl[j * nin + k];
#pragma unroll
        for (int q = 0; q < 16; ++q) accv[q] += w * act[pg * 16 + q][k];
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) nxt[pg * 16 + q][j] = last ? accv[q] : tanhf(accv[q]);
    }
    __syncthreads();
    for (int u = t; u < kTrunkPix * 128; u += 256) act[u >> 7][u & 127] = nxt[u >> 7][u & 127];
    __syncthreads();
    nin = nout;
  }
  // fold the head: C0 + 1 outputs per pixel
  const float* Wh = params + td.oWh;  // [basis][C0]
  const float* bh = params + td.obh;  // [basis]
  const int nf = td.c0 + 1;
  for (int u = t; u < kTrunkPix * nf; u += 256) {
    const int q = u / nf, c = u - q * nf;
    const int64_t p = p0 + q;
    if (p >= npix) continue;
    float s = 0.f;
    for (int k = 0; k < td.basis; ++k) s += (c < td.c0 ? Wh[k * td.c0 + c] : bh[k]) * act[q][k];
    out[p * td.fold_pitch + c] = s;
  }
}

// ---------------------------------------------------------------------------
// Static channels of the activation buffers: normalised widths (hx, hy) at
// channel `coff`, and optionally the mask at channel `moff` (level 0 input).
__global__ void k_fill_static(int H, int W, int pitch, int coff, const float* __restrict__ hxn,
                              const float* __restrict__ hyn, const uint8_t* __restrict__ mask, int moff,
                              bf16_t* __restrict__ buf, int64_t bstride) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)H * W) return;
  const int j = (int)(p / W), i = (int)(p - (int64_t)j * W);
  bf16_t* b = buf + blockIdx.y * bstride + p * pitch;
  if (coff >= 0) {
    b[coff] = f2bf(hxn[i]);
    b[coff + 1] = f2bf(hyn[j]);
  }
  if (moff >= 0) b[moff] = f2bf(mask ? (float)mask[p] : 0.f);
}

// Partial sums of r^2 per workgroup (fixed grid of kRedBlocks per sample).
template <bool GRP>
__global__ __launch_bounds__(256) void k_sumsq(const float* __restrict__ r, int64_t n, double* __restrict__ part,
                                               const PackMember* __restrict__ mem) {
  __shared__ double lds[kWaves];
  int smp = blockIdx.y;
  if constexpr (GRP) {
    const PackMember& M = mem[blockIdx.y];
    if (M.skip && *M.skip != 0) return;
    r = M.r;
    n = M.n;
    part = M.part;
    smp = 0;
  }
  const float* rs = r + (int64_t)smp * n;
  double s = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) {
    const double v = rs[k];
    s += v * v;
  }
  s = block_sum(s, lds);
  if (threadIdx.x == 0) part[smp * gridDim.x + blockIdx.x] = s;
}

// Channel 0 of the level-0 input: r * sqrt(N) / ||r|| in BF16 (0 for r = 0).
// ||r||^2 comes from the kRedBlocks partials of k_sumsq, reduced in the same
// order by every workgroup.
template <bool GRP>
__global__ __launch_bounds__(256) void k_input_pack(const float* __restrict__ r, int64_t n, const double* __restrict__ part,
                                                    int nparts, bf16_t* __restrict__ xin, int pitch, int64_t bstride,
                                                    const PackMember* __restrict__ mem) {
  __shared__ double lds[kWaves];
  int smp = blockIdx.y;
  if constexpr (GRP) {
    const PackMember& M = mem[blockIdx.y];
    if (M.skip && *M.skip != 0) return;
    r = M.r;
    n = M.n;
    part = M.part;
    xin = M.xin;
    smp = 0;
  }
  const double rr = reduce_partials(part + (int64_t)smp * nparts, nparts, lds);
  const float scale = rr > 0.0 ? (float)(sqrt((double)n) / sqrt(rr)) : 0.f;
  const float* rs = r + (int64_t)smp * n;
  bf16_t* xs = xin + (int64_t)smp * bstride;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256)
    xs[k * pitch] = f2bf(rs[k] * scale);
}

// 2x2 average pooling of C channels (8 per thread) from a buffer of pitch
// pin at channel offset cin_off into a buffer of pitch pout (channel 0 on).
__global__ void k_pool2(int Ho, int Wo, int C, const bf16_t* __restrict__ in, int pin, int cin_off, int64_t in_bs,
                        bf16_t* __restrict__ out, int pout, int64_t out_bs) {
  const int smp = blockIdx.y;
  const int c8n = C / 8;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)Ho * Wo * c8n) return;
  const int c8 = (int)(idx % c8n);
  const int64_t p = idx / c8n;
  const int yo = (int)(p / Wo), xo = (int)(p - (int64_t)yo * Wo);
  const int Wi = 2 * Wo;
  const bf16_t* ib = in + smp * in_bs + cin_off + c8 * 8;
  float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const uint4 v = *(const uint4*)(ib + ((size_t)(2 * yo + a) * Wi + 2 * xo + b) * pin);
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        s[2 * q] += bf2f((bf16_t)(w[q] & 0xffff));
        s[2 * q + 1] += bf2f((bf16_t)(w[q] >> 16));
      }
    }
  uint32_t o[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) o[q] = (uint32_t)f2bf(0.25f * s[2 * q]) | ((uint32_t)f2bf(0.25f * s[2 * q + 1]) << 16);
  *(uint4*)(out + smp * out_bs + p * pout + c8 * 8) = make_uint4(o[0], o[1], o[2], o[3]);
}

// DeepONet output y = gamma * (D0 . fold[p][0:C0] + fold[p][C0]) in FP32.
// Eight lanes per pixel, lane l taking channels 4l + 32k, so that a pixel's
// D0 and fold rows are read contiguously (fold rows are padded to a multiple
// of 4 floats); the eight partial sums are added with lane shuffles.
template <bool GRP>
__global__ void k_deeponet_out(int64_t npix, int c0, const bf16_t* __restrict__ d0, int64_t d_bs,
                               const float* __restrict__ fold, int fold_pitch, const float* __restrict__ gamma,
                               float* __restrict__ y, const OutMember* __restrict__ mem) {
  int smp = blockIdx.y;
  if constexpr (GRP) {
    const OutMember& M = mem[blockIdx.y];
    if (M.skip && *M.skip != 0) return;
    npix = M.npix;
    d0 = M.d0;
    fold = M.fold;
    y = M.y;
    smp = 0;
  }
  const int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const int l = threadIdx.x & 7;
  float s = 0.f;
  if (p < npix) {
    const bf16_t* d = d0 + smp * d_bs + p * c0;
    const float* f = fold + p * fold_pitch;
    for (int c = 4 * l; c < c0; c += 32) s += out_group4(*(const uint2*)(d + c), *(const float4*)(f + c));
  }
  s += __shfl_xor(s, 4, 8);
  s += __shfl_xor(s, 2, 8);
  s += __shfl_xor(s, 1, 8);
  if (p < npix && l == 0) y[smp * npix + p] = gamma[0] * (s + fold[p * fold_pitch + c0]);
}

// ---------------------------------------------------------------------------
// Launchers.
// Compute units of the current device (256 on MI355X), queried once.
static int conv_device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      cus = n;
    else
      cus = 256;
  }
  return cus;
}

// Room for the partial sums of any split layer: a layer splits only with
// tiles * cot * nb < cus workgroups, into ks <= ceil(cus / (tiles * cot * nb))
// shares, so ks * nb * pixels * channel pitch < 2 * cus * 256 * 64.
int64_t conv_kpart_elems() { return (int64_t)2 * conv_device_cus() * kCTH * kCTW * 64; }

// Resident workgroups per CU of a convolution kernel (registers and LDS),
// queried once per instantiation.
template <int TN, int TAPS, bool UP, int ETA, bool WSTAT, bool GRP, bool XU = false, bool OUTF = false>
static int conv_per_cu() {
  static int per_cu = 0;
  if (per_cu == 0) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_conv<TN, TAPS, UP, ETA, WSTAT, GRP, XU, OUTF>, 256, 0) !=
            hipSuccess ||
        n < 1)
      n = 1;
    per_cu = n;
  }
  return per_cu;
}

// Small 1x1 layers (at most 128 input and output channels, one input source,
// no local weight, upsampling or pooling) run as the skinny GEMM.
static bool conv_skinny(int taps, bool up, bool has_eta, const ConvGeo& g, int Kp) {
  return taps == 1 && !up && !has_eta && !g.x1 && !g.xu && !g.pool_y && g.cout <= 128 && Kp <= 128 &&
         g.y_pitch % 8 == 0 && g.y_off % 8 == 0;
}

static int conv_tiles(const ConvGeo& g) { return ((g.W + kCTW - 1) / kCTW) * ((g.H + kCTH - 1) / kCTH); }

// K shares of a layer's launch over nb samples with tn output channels per
// workgroup. Layers with fewer workgroups than compute units (the coarse
// levels of small grids) split their nch chunks of input channels over up to
// ceil(cus / workgroups) workgroups, when the caller gave room for the
// partials (cp: the channel pitch of the launch's partials). A grouped launch
// applies the same rule to each member alone, with the member's own tn, so
// that a member's sums are those of its own launch.
static int conv_ksplit(const ConvGeo& g, int nb, int tn, int nch, bool have_kpart, int64_t kpart_elems, int cp) {
  const int cot = (g.cout + tn - 1) / tn;
  const int cus = conv_device_cus();
  const int64_t wgs = (int64_t)conv_tiles(g) * cot * nb;
  int ks = 1;
  if (have_kpart && wgs < cus && nch > 1 && g.cout % 4 == 0) {
    ks = (int)std::min<int64_t>(nch, (cus + wgs - 1) / wgs);
    const int cps = (nch + ks - 1) / ks;
    ks = (nch + cps - 1) / cps;  // no empty shares
    if ((int64_t)ks * nb * g.H * g.W * cp > kpart_elems) ks = 1;
  }
  return ks;
}

// Output channels per workgroup by default: 64 when the layer has at least
// 64 output channels and still at least two workgroups per compute unit with
// them (each staged input chunk then serves twice the channels), else 32
// (twice the workgroups). Measured per layer on 64^2 to 1024^2 grids, the
// wider tile won only above that count.
int conv_default_tile(const ConvGeo& g, int nb) {
  if (g.cout < 64) return 32;
  const int64_t wgs64 = (int64_t)conv_tiles(g) * ((g.cout + 63) / 64) * nb;
  return wgs64 >= 2 * (int64_t)conv_device_cus() ? 64 : 32;
}

template <int TN, int TAPS, bool UP, int ETA>
static void conv_go_eta(const ConvGeo& g, int nb, const bf16_t* x, const bf16_t* eta, const bf16_t* wp, int Kp,
                        const float* bias, bf16_t* y, hipStream_t s, float* kpart, int64_t kpart_elems) {
  const int tiles = conv_tiles(g);
  const int cot = (g.cout + TN - 1) / TN;
  const int cus = conv_device_cus();
  const int64_t wgs = (int64_t)tiles * cot * nb;
  const int nch = (g.cin8 + ConvShape<TN, TAPS>::CK - 1) / ConvShape<TN, TAPS>::CK;
  const int ks = conv_ksplit(g, nb, TN, nch, kpart != nullptr, kpart_elems, cot * TN);
  // one chunk per workgroup: the weight slice is staged once
  const bool wstat = (nch + ks - 1) / ks == 1;
  // runs of tiles that fill the resident workgroups once
  const int per_cu =
      wstat ? conv_per_cu<TN, TAPS, UP, ETA, true, false>() : conv_per_cu<TN, TAPS, UP, ETA, false, false>();
  const int64_t slots = (int64_t)cus * per_cu;
  const int run = (int)std::max<int64_t>(1, (wgs + slots - 1) / slots);
  const dim3 grid((tiles + run - 1) / run, cot, nb * ks);
  // the coarse input source only in the kernels of layers that have one
  bool launched = false;
  if constexpr (TAPS == 9 && !UP) {
    if (g.xu) {
      if (wstat)
        k_conv<TN, TAPS, UP, ETA, true, false, true><<<grid, 256, 0, s>>>(g, x, eta, wp, Kp, bias, y, run, kpart, ks,
                                                                          nullptr, 0, OutFold{});
      else
        k_conv<TN, TAPS, UP, ETA, false, false, true><<<grid, 256, 0, s>>>(g, x, eta, wp, Kp, bias, y, run, kpart, ks,
                                                                           nullptr, 0, OutFold{});
      launched = true;
    }
  }
  if (!launched) {
    if (wstat)
      k_conv<TN, TAPS, UP, ETA, true, false, false><<<grid, 256, 0, s>>>(g, x, eta, wp, Kp, bias, y, run, kpart, ks,
                                                                         nullptr, 0, OutFold{});
    else
      k_conv<TN, TAPS, UP, ETA, false, false, false><<<grid, 256, 0, s>>>(g, x, eta, wp, Kp, bias, y, run, kpart, ks,
                                                                          nullptr, 0, OutFold{});
  }
  if (ks > 1) {
    const int64_t n = (int64_t)g.H * g.W * (g.cout / 4);
    k_conv_ksum<UP, false><<<dim3((unsigned)((n + 255) / 256), nb), 256, 0, s>>>(g, nb, ks, cot * TN, kpart, bias, y,
                                                                                 nullptr);
  }
}

// Grouped convolution: the members' K splits and runs of tiles, one launch
// shape for all of them (runs of tiles that fill the resident workgroups once
// over the whole group).
template <int TN, int TAPS, bool UP, int ETA>
static void conv_group_plan_t(std::vector<ConvMember>& m, int64_t kpart_elems, ConvGroupLaunch& L) {
  const ConvGeo& g0 = m[0].g;
  const int cot = (g0.cout + TN - 1) / TN;
  const int nch = (g0.cin8 + ConvShape<TN, TAPS>::CK - 1) / ConvShape<TN, TAPS>::CK;
  int64_t wgs = 0, kwg = 0;
  bool wstat = true;
  for (ConvMember& e : m) {
    // the K split of the member's own launch (its own tile width)
    e.ks = conv_ksplit(e.g, 1, e.tn ? e.tn : conv_default_tile(e.g, 1), nch, e.kpart != nullptr, kpart_elems,
                       cot * TN);
    wgs += (int64_t)conv_tiles(e.g) * cot * e.ks;
    wstat = wstat && (nch + e.ks - 1) / e.ks == 1;
    e.kwg0 = (int)kwg;
    if (e.ks > 1) kwg += ((int64_t)e.g.H * e.g.W * (e.g.cout / 4) + 255) / 256;
  }
  const int per_cu =
      wstat ? conv_per_cu<TN, TAPS, UP, ETA, true, true>() : conv_per_cu<TN, TAPS, UP, ETA, false, true>();
  L.xu = m[0].g.xu != nullptr;
  const int64_t slots = (int64_t)conv_device_cus() * per_cu;
  const int run = (int)std::max<int64_t>(1, (wgs + slots - 1) / slots);
  int64_t wg = 0;
  for (ConvMember& e : m) {
    e.nwt = (conv_tiles(e.g) + run - 1) / run;
    e.wg0 = (int)wg;
    wg += (int64_t)e.nwt * e.ks;
  }
  L.tn = TN;
  L.wstat = wstat;
  L.run = run;
  L.gx = (int)wg;
  L.cot = cot;
  L.nmem = (int)m.size();
  L.split = kwg > 0;
  L.ksum_gx = (int)kwg;
}

template <int TN, int TAPS, bool UP, int ETA>
static void conv_group_launch_t(const ConvGroupLaunch& L, const ConvMember* dm, const bf16_t* wp, int Kp,
                                const float* bias, hipStream_t s) {
  const ConvGeo g0{};
  const dim3 grid(L.gx, L.cot, 1);
  bool launched = false;
  if constexpr (TAPS == 9 && !UP) {
    if (L.xu) {
      if (L.wstat)
        k_conv<TN, TAPS, UP, ETA, true, true, true><<<grid, 256, 0, s>>>(g0, nullptr, nullptr, wp, Kp, bias, nullptr,
                                                                         L.run, nullptr, 1, dm, L.nmem, OutFold{});
      else
        k_conv<TN, TAPS, UP, ETA, false, true, true><<<grid, 256, 0, s>>>(g0, nullptr, nullptr, wp, Kp, bias, nullptr,
                                                                          L.run, nullptr, 1, dm, L.nmem, OutFold{});
      launched = true;
    }
  }
  if (!launched) {
    if (L.wstat)
      k_conv<TN, TAPS, UP, ETA, true, true, false><<<grid, 256, 0, s>>>(g0, nullptr, nullptr, wp, Kp, bias, nullptr,
                                                                        L.run, nullptr, 1, dm, L.nmem, OutFold{});
    else
      k_conv<TN, TAPS, UP, ETA, false, true, false><<<grid, 256, 0, s>>>(g0, nullptr, nullptr, wp, Kp, bias, nullptr,
                                                                         L.run, nullptr, 1, dm, L.nmem, OutFold{});
  }
  if (L.split)
    k_conv_ksum<UP, true><<<dim3(L.ksum_gx, 1), 256, 0, s>>>(g0, L.nmem, 1, L.cot * TN, nullptr, bias, nullptr, dm);
}

// The instantiations a grouped forward uses: 3x3 layers with any local
// weight, and 1x1 layers without one.
template <class F>
static bool conv_group_dispatch(int taps, bool up, int eta, bool wide, F&& f) {
  using std::integral_constant;
  auto by_eta = [&](auto tn, auto tp, auto upc) {
    if (eta == kEtaNone) f(tn, tp, upc, integral_constant<int, kEtaNone>{});
    else if (eta == kEtaNode) f(tn, tp, upc, integral_constant<int, kEtaNode>{});
    else f(tn, tp, upc, integral_constant<int, kEtaChannel>{});
  };
  if (taps == 9 && !up) {
    if (wide) by_eta(integral_constant<int, 64>{}, integral_constant<int, 9>{}, integral_constant<bool, false>{});
    else by_eta(integral_constant<int, 32>{}, integral_constant<int, 9>{}, integral_constant<bool, false>{});
    return true;
  }
  if (taps == 1 && eta == kEtaNone) {
    const auto none = integral_constant<int, kEtaNone>{};
    if (up) {
      if (wide) f(integral_constant<int, 64>{}, integral_constant<int, 1>{}, integral_constant<bool, true>{}, none);
      else f(integral_constant<int, 32>{}, integral_constant<int, 1>{}, integral_constant<bool, true>{}, none);
    } else {
      if (wide) f(integral_constant<int, 64>{}, integral_constant<int, 1>{}, integral_constant<bool, false>{}, none);
      else f(integral_constant<int, 32>{}, integral_constant<int, 1>{}, integral_constant<bool, false>{}, none);
    }
    return true;
  }
  return false;
}

static int conv_eta_mode(const ConvMember& e) { return !e.eta ? kEtaNone : e.g.eta_node ? kEtaNode : kEtaChannel; }

bool plan_conv_group(int taps, bool up, int Kp, std::vector<ConvMember>& m, int64_t kpart_elems,
                     ConvGroupLaunch& L) {
  if (m.empty()) return false;
  L = ConvGroupLaunch{};
  L.taps = taps;
  L.up = up;
  L.eta = conv_eta_mode(m[0]);
  if (conv_skinny(taps, up, m[0].eta != nullptr, m[0].g, Kp)) {
    // the skinny GEMM of each member, blockIdx.y the member: its own launch's
    // runs of workgroups, the largest over the members
    L.skinny = m[0].g.cout <= 32 ? 2 : m[0].g.cout <= 64 ? 4 : 8;
    L.nmem = (int)m.size();
    int per_cu = 1;
    const auto fn = L.skinny == 2 ? k_conv1x1<2, true> : L.skinny == 4 ? k_conv1x1<4, true> : k_conv1x1<8, true>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0) != hipSuccess || per_cu < 1) per_cu = 1;
    const int64_t want = (int64_t)conv_device_cus() * per_cu;
    for (const ConvMember& e : m) {
      const int tiles = (e.g.H * e.g.W + 15) / 16;
      L.gx = std::max(L.gx, (int)std::max<int64_t>(1, std::min<int64_t>((tiles + 3) / 4, want / L.nmem)));
    }
    return true;
  }
  // the group's tile width by the default rule over all members' workgroups
  bool wide = false;
  if (m[0].g.cout >= 64) {
    int64_t wgs64 = 0;
    for (const ConvMember& e : m) wgs64 += (int64_t)conv_tiles(e.g) * ((e.g.cout + 63) / 64);
    wide = wgs64 >= 2 * (int64_t)conv_device_cus();
  }
  return conv_group_dispatch(taps, up, L.eta, wide, [&](auto tn, auto tp, auto upc, auto et) {
    conv_group_plan_t<decltype(tn)::value, decltype(tp)::value, decltype(upc)::value, decltype(et)::value>(
        m, kpart_elems, L);
  });
}

void launch_conv_group(const ConvGroupLaunch& L, const ConvMember* d_mem, const bf16_t* wp, int Kp,
                       const float* bias, hipStream_t s) {
  if (L.skinny) {
    const ConvGeo g0{};
    const dim3 grid(L.gx, L.nmem);
    if (L.skinny == 2) k_conv1x1<2, true><<<grid, 256, 0, s>>>(g0, nullptr, wp, Kp, bias, nullptr, d_mem);
    else if (L.skinny == 4) k_conv1x1<4, true><<<grid, 256, 0, s>>>(g0, nullptr, wp, Kp, bias, nullptr, d_mem);
    else k_conv1x1<8, true><<<grid, 256, 0, s>>>(g0, nullptr, wp, Kp, bias, nullptr, d_mem);
    return;
  }
  conv_group_dispatch(L.taps, L.up, L.eta, L.tn == 64, [&](auto tn, auto tp, auto upc, auto et) {
    conv_group_launch_t<decltype(tn)::value, decltype(tp)::value, decltype(upc)::value, decltype(et)::value>(
        L, d_mem, wp, Kp, bias, s);
  });
}

template <int TN, int TAPS, bool UP>
static void conv_go(const ConvGeo& g, int nb, const bf16_t* x, const bf16_t* eta, const bf16_t* wp, int Kp,
                    const float* bias, bf16_t* y, hipStream_t s, float* kpart, int64_t kpart_elems) {
  if (!eta)
    conv_go_eta<TN, TAPS, UP, kEtaNone>(g, nb, x, eta, wp, Kp, bias, y, s, kpart, kpart_elems);
  else if (g.eta_node)
    conv_go_eta<TN, TAPS, UP, kEtaNode>(g, nb, x, eta, wp, Kp, bias, y, s, kpart, kpart_elems);
  else
    conv_go_eta<TN, TAPS, UP, kEtaChannel>(g, nb, x, eta, wp, Kp, bias, y, s, kpart, kpart_elems);
}

template <int MT>
static void conv1x1_go(const ConvGeo& g, int nb, const bf16_t* x, const bf16_t* wp, int Kp, const float* bias,
                       bf16_t* y, hipStream_t s) {
  static int per_cu = 0;
  if (per_cu == 0) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_conv1x1<MT, false>, 256, 0) != hipSuccess || n < 1) n = 1;
    per_cu = n;
  }
  const int tiles = (g.H * g.W + 15) / 16;
  const int64_t want = (int64_t)conv_device_cus() * per_cu;
  const int per_smp = (int)std::max<int64_t>(1, std::min<int64_t>((tiles + 3) / 4, want / nb));
  k_conv1x1<MT, false><<<dim3(per_smp, nb), 256, 0, s>>>(g, x, wp, Kp, bias, y, nullptr);
}

// The last decoder convolution with the DeepONet output in its epilogue
// (one launch of 32 output channels per workgroup, no K split).
template <int ETA>
static void conv_out_go(const ConvGeo& g, int nb, const bf16_t* x, const bf16_t* eta, const bf16_t* wp, int Kp,
                        const float* bias, bf16_t* y, int nch, const OutFold& of, hipStream_t s) {
  const int tiles = conv_tiles(g);
  const bool wstat = nch == 1;
  const int per_cu = wstat ? conv_per_cu<32, 9, false, ETA, true, false, false, true>()
                           : conv_per_cu<32, 9, false, ETA, false, false, false, true>();
  const int64_t slots = (int64_t)conv_device_cus() * per_cu;
  const int run = (int)std::max<int64_t>(1, ((int64_t)tiles * nb + slots - 1) / slots);
  const dim3 grid((tiles + run - 1) / run, 1, nb);
  if (wstat)
    k_conv<32, 9, false, ETA, true, false, false, true><<<grid, 256, 0, s>>>(g, x, eta, wp, Kp, bias, y, run, nullptr,
                                                                              1, nullptr, 0, of);
  else
    k_conv<32, 9, false, ETA, false, false, false, true><<<grid, 256, 0, s>>>(g, x, eta, wp, Kp, bias, y, run, nullptr,
                                                                               1, nullptr, 0, of);
}

bool launch_conv_out(const ConvGeo& g, int nb, const bf16_t* x, const bf16_t* eta, const bf16_t* wp, int Kp,
                     const float* bias, bf16_t* y, hipStream_t s, float* kpart, int64_t kpart_elems, int tn,
                     const OutFold& of) {
  if (g.xu || g.pool_y || g.cout != of.c0 || of.c0 > 32 || of.c0 % 4 || of.pitch % 4 || !of.fold || !of.y ||
      (tn ? tn : conv_default_tile(g, nb)) != 32)
    return false;
  const int nch = (g.cin8 + ConvShape<32, 9>::CK - 1) / ConvShape<32, 9>::CK;
  if (conv_ksplit(g, nb, 32, nch, kpart != nullptr, kpart_elems, 32) > 1) return false;
  if (!eta)
    conv_out_go<kEtaNone>(g, nb, x, eta, wp, Kp, bias, y, nch, of, s);
  else if (g.eta_node)
    conv_out_go<kEtaNode>(g, nb, x, eta, wp, Kp, bias, y, nch, of, s);
  else
    conv_out_go<kEtaChannel>(g, nb, x, eta, wp, Kp, bias, y, nch, of, s);
  return true;
}

bool conv_has_tile_choice(int taps, bool up, bool has_eta, const ConvGeo& g, int Kp) {
  return !conv_skinny(taps, up, has_eta, g, Kp) && g.cout >= 64;
}

void launch_conv(int taps, bool up, const ConvGeo& g, int nb, const bf16_t* x, const bf16_t* eta, const bf16_t* wp,
                 int Kp, const float* bias, bf16_t* y, hipStream_t s, float* kpart, int64_t kpart_elems, int tn) {
  if (conv_skinny(taps, up, eta != nullptr, g, Kp)) {
    // small 1x1 layers: the skinny GEMM, one round of resident workgroups
    // over all samples
    if (g.cout <= 32) conv1x1_go<2>(g, nb, x, wp, Kp, bias, y, s);
    else if (g.cout <= 64) conv1x1_go<4>(g, nb, x, wp, Kp, bias, y, s);
    else conv1x1_go<8>(g, nb, x, wp, Kp, bias, y, s);
    return;
  }
  const bool wide = (tn ? tn : conv_default_tile(g, nb)) == 64;
  if (taps == 9) {
    if (wide) conv_go<64, 9, false>(g, nb, x, eta, wp, Kp, bias, y, s, kpart, kpart_elems);
    else conv_go<32, 9, false>(g, nb, x, eta, wp, Kp, bias, y, s, kpart, kpart_elems);
  } else if (up) {
    if (wide) conv_go<64, 1, true>(g, nb, x, eta, wp, Kp, bias, y, s, kpart, kpart_elems);
    else conv_go<32, 1, true>(g, nb, x, eta, wp, Kp, bias, y, s, kpart, kpart_elems);
  } else {
    if (wide) conv_go<64, 1, false>(g, nb, x, eta, wp, Kp, bias, y, s, kpart, kpart_elems);
    else conv_go<32, 1, false>(g, nb, x, eta, wp, Kp, bias, y, s, kpart, kpart_elems);
  }
}

void launch_pack_weights(const float* w, int cout, int cin, int cin8, int taps, int Kp, bf16_t* out, hipStream_t s) {
  const int64_t n = (int64_t)cout * Kp;
  k_pack_weights<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(w, cout, cin8, taps, Kp, 0, cout, cin, out);
}

void launch_pack_weights_t(const float* w, int cout_fwd, int cin_fwd, int rows, int taps, int Kp, bf16_t* out,
                           hipStream_t s) {
  const int64_t n = (int64_t)rows * Kp;
  k_pack_weights<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(w, rows, cout_fwd, taps, Kp, 1, cout_fwd, cin_fwd, out);
}

void launch_eta(int H, int W, int cin, int cin8, int hid, const float* dxl, const float* dxr, const float* dyd,
                const float* dyu, const float* W1, const float* b1, const float* W2, const float* b2, bf16_t* eta,
                hipStream_t s) {
  const int64_t n = (int64_t)H * W;
  k_eta<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(H, W, cin, cin8, hid, dxl, dxr, dyd, dyu, W1, b1, W2, b2, eta);
}

void launch_trunk_fold(int H, int W, const float* xin, const float* yin, const float* params, const TrunkDesc& td,
                       float* out, hipStream_t s) {
  const int64_t n = (int64_t)H * W;
  k_trunk_fold<<<(unsigned)((n + kTrunkPix - 1) / kTrunkPix), 256, 0, s>>>(H, W, xin, yin, params, td, out);
}

void launch_fill_static(int H, int W, int pitch, int coff, const float* hxn, const float* hyn, const uint8_t* mask,
                        int moff, bf16_t* buf, int64_t bstride, int nb, hipStream_t s) {
  const int64_t n = (int64_t)H * W;
  k_fill_static<<<dim3((unsigned)((n + 255) / 256), nb), 256, 0, s>>>(H, W, pitch, coff, hxn, hyn, mask, moff, buf,
                                                                       bstride);
}

void launch_sumsq(const float* r, int64_t n, int nb, double* part, hipStream_t s) {
  k_sumsq<false><<<dim3(kRedBlocks, nb), 256, 0, s>>>(r, n, part, nullptr);
}

void launch_input_pack(const float* r, int64_t n, int nb, double* part, bf16_t* xin, int pitch, int64_t bstride,
                       hipStream_t s) {
  k_sumsq<false><<<dim3(kRedBlocks, nb), 256, 0, s>>>(r, n, part, nullptr);
  k_input_pack<false><<<dim3(kRedBlocks, nb), 256, 0, s>>>(r, n, part, kRedBlocks, xin, pitch, bstride, nullptr);
}

void launch_pool2(int Ho, int Wo, int C, const bf16_t* in, int pin, int cin_off, int64_t in_bs, bf16_t* out, int pout,
                  int64_t out_bs, int nb, hipStream_t s) {
  const int64_t n = (int64_t)Ho * Wo * (C / 8);
  k_pool2<<<dim3((unsigned)((n + 255) / 256), nb), 256, 0, s>>>(Ho, Wo, C, in, pin, cin_off, in_bs, out, pout, out_bs);
}

void launch_input_pack_group(const PackMember* d_mem, int n, int pitch, hipStream_t s) {
  k_sumsq<true><<<dim3(kRedBlocks, n), 256, 0, s>>>(nullptr, 0, nullptr, d_mem);
  k_input_pack<true><<<dim3(kRedBlocks, n), 256, 0, s>>>(nullptr, 0, nullptr, kRedBlocks, nullptr, pitch, 0, d_mem);
}

void launch_deeponet_out_group(const OutMember* d_mem, int n, int64_t max_npix, int c0, int fold_pitch,
                               const float* gamma, hipStream_t s) {
  k_deeponet_out<true><<<dim3((unsigned)((max_npix * 8 + 255) / 256), n), 256, 0, s>>>(
      0, c0, nullptr, 0, nullptr, fold_pitch, gamma, nullptr, d_mem);
}

void launch_deeponet_out(int64_t npix, int c0, const bf16_t* d0, int64_t d_bs, const float* fold, int fold_pitch,
                         const float* gamma, float* y, int nb, hipStream_t s) {
  k_deeponet_out<false><<<dim3((unsigned)((npix * 8 + 255) / 256), nb), 256, 0, s>>>(npix, c0, d0, d_bs, fold,
                                                                                  fold_pitch, gamma, y, nullptr);
}

}  // namespace ppe
