// Training kernels of the DeepONet: weight gradients on BF16 MFMA (split-K
// over pixels, fixed-order reduction), activation-gradient masks, the
// Mesh-Conv local-weight backward, pooling / upsampling / concatenation
// backward, the DeepONet contraction, the residual loss of Eq. 19, and Adam.
#include <algorithm>

#include "common.hpp"
#include "net_common.hpp"
#include "net_kernels.hpp"
#include "train_kernels.hpp"

namespace ppe {

// ---------------------------------------------------------------------------
// Weight gradient of a convolution layer:
//   dW[co][ci][tap] = sum over pixels p of dPre[p][co] * Xbar[p + off(tap)][ci]
// with Xbar = eta * X (the layer's weighted input). MFMA 16x16x32 BF16 with
// A = dPre^T (M = 32 output channels per workgroup, K = pixels) and
// B = shifted Xbar (N = 32 input channels per workgroup). Wave w owns the
// (co, ci) sub-tile (w / 2, w % 2) for all taps. Each workgroup (split z)
// accumulates 8 x 16 pixel tiles z, z + nsplit, ... of all samples and writes
// its partial sums in the master layout [co][ci < cin][tap]; k_reduce_rows
// sums the splits in a fixed order.
__device__ __forceinline__ void transpose8x8_bf16(const uint4 (&v)[8], uint4 (&w)[8]) {
  // v[r] holds channels 0..7 of pixel r; w[e] receives pixels 0..7 of channel e
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    uint32_t o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint4 a4 = v[2 * j], b4 = v[2 * j + 1];
      const uint32_t a = (e / 2 == 0) ? a4.x : (e / 2 == 1) ? a4.y : (e / 2 == 2) ? a4.z : a4.w;
      const uint32_t b = (e / 2 == 0) ? b4.x : (e / 2 == 1) ? b4.y : (e / 2 == 2) ? b4.z : b4.w;
      o[j] = (e & 1) ? ((a >> 16) | (b & 0xffff0000u)) : ((a & 0xffffu) | (b << 16));
    }
    w[e] = make_uint4(o[0], o[1], o[2], o[3]);
  }
}

template <int TAPS>
__global__ __launch_bounds__(256) void k_wgrad(WgradGeo g, const bf16_t* __restrict__ dp, const bf16_t* __restrict__ x,
                                               const bf16_t* __restrict__ eta, float* __restrict__ part) {
  constexpr int HALO = TAPS == 9 ? 1 : 0;
  constexpr int TH = 8, TW = 16, NP = TH * TW;
  constexpr int LH = TH + 2 * HALO;
  constexpr int NDX = TAPS == 9 ? 3 : 1;
  constexpr int DPP = NP + 8;   // LDS pitch of a transposed dPre row
  constexpr int XPP = TW + 8;   // LDS pitch of a staged input row
  constexpr int CIP = LH * XPP + 8;  // LDS pitch of one input channel's rows (16 lanes in distinct banks)
  // staging units of 8 pixels x 8 channels, each loaded with 16-byte loads,
  // transposed in registers and written as 16-byte LDS rows: dPre (4 channel
  // groups x 16 pixel octets), then the weighted input (NDX column shifts x 4
  // channel groups x LH rows x 2 column octets)
  constexpr int NUD = 4 * (NP / 8), NUXS = NDX * 4 * LH * (TW / 8);
  constexpr int NUS = NUD + NUXS, RND = (NUS + 255) / 256;
  __shared__ __attribute__((aligned(16))) bf16_t s_dp[32 * DPP];
  __shared__ __attribute__((aligned(16))) bf16_t s_x[NDX * 32 * CIP];
  const int co0 = blockIdx.x * 32, ci0 = blockIdx.y * 32;
  const int split = blockIdx.z, nsplit = gridDim.z;
  const int tiles_x = (g.W + TW - 1) / TW, tiles_y = (g.H + TH - 1) / TH;
  const int tiles = tiles_x * tiles_y * g.nb;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int mt = wv >> 1, nt = wv & 1;
  f32x4_t acc[TAPS];
#pragma unroll
  for (int t = 0; t < TAPS; ++t) acc[t] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  for (int t = split; t < tiles; t += nsplit) {
    const int smp = t / (tiles_x * tiles_y);
    const int rem = t - smp * tiles_x * tiles_y;
    const int py0 = (rem / tiles_x) * TH, px0 = (rem % tiles_x) * TW;
    const bf16_t* dps = dp + (int64_t)smp * g.dp_bstride;
    const bf16_t* xs = x + (int64_t)smp * g.x_bstride;
    const bf16_t* es = eta ? eta + (int64_t)smp * g.e_bstride : nullptr;
    __syncthreads();  // the previous tile's MFMA loop is done with LDS
#pragma unroll
    for (int rd = 0; rd < RND; ++rd) {
      const int u = threadIdx.x + 256 * rd;
      if (u >= NUS) continue;
      uint4 v[8], w[8];
      if (u < NUD) {
        // dPre: channel group cg of pixels 8 oct .. 8 oct + 7 (one tile row)
        const int cg = u & 3, oct = u >> 2;
        const int py = py0 + (oct * 8) / TW, pxb = px0 + (oct * 8) % TW;
        const bool ok = py < g.H && co0 + cg * 8 < g.cout;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          v[r] = make_uint4(0, 0, 0, 0);
          if (ok && pxb + r < g.W)
            v[r] = *(const uint4*)(dps + ((int64_t)py * g.W + pxb + r) * g.dp_pitch + co0 + cg * 8);
        }
        transpose8x8_bf16(v, w);
#pragma unroll
        for (int e = 0; e < 8; ++e) *(uint4*)(s_dp + (cg * 8 + e) * DPP + oct * 8) = w[e];
      } else {
        // weighted input, column shift dx: s_x[dx][ci][row][col] = Xbar[row - H][col + dx - H]
        const int q = u - NUD;
        const int oct = q & 1;
        int r2 = q >> 1;
        const int row = r2 % LH;
        r2 /= LH;
        const int cg = r2 % 4, dx = r2 / 4;
        const int gy = py0 + row - HALO, gxb = px0 + oct * 8 + dx - HALO;
        const bool ok = gy >= 0 && gy < g.H && ci0 + cg * 8 < g.cin8;
        uint4 ev[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          v[r] = make_uint4(0, 0, 0, 0);
          ev[r] = make_uint4(0, 0, 0, 0);
          const int gx = gxb + r;
          if (ok && gx >= 0 && gx < g.W) {
            const int64_t pix = (int64_t)gy * g.W + gx;
            const int64_t off = pix * g.cin8 + ci0 + cg * 8;
            v[r] = *(const uint4*)(xs + off);
            if (es) {
              if (g.eta_node) {  // one weight for the pixel's eight channels
                const uint32_t e2 = (uint32_t)es[pix] * 0x10001u;
                ev[r] = make_uint4(e2, e2, e2, e2);
              } else {
                ev[r] = *(const uint4*)(es + off);
              }
            }
          }
        }
        if (es) {
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            const uint32_t a4[4] = {v[r].x, v[r].y, v[r].z, v[r].w}, b4[4] = {ev[r].x, ev[r].y, ev[r].z, ev[r].w};
            uint32_t o4[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const float lo = bf2f((bf16_t)(a4[k] & 0xffff)) * bf2f((bf16_t)(b4[k] & 0xffff));
              const float hi = bf2f((bf16_t)(a4[k] >> 16)) * bf2f((bf16_t)(b4[k] >> 16));
              o4[k] = (uint32_t)f2bf(lo) | ((uint32_t)f2bf(hi) << 16);
            }
            v[r] = make_uint4(o4[0], o4[1], o4[2], o4[3]);
          }
        }
        transpose8x8_bf16(v, w);
#pragma unroll
        for (int e = 0; e < 8; ++e) *(uint4*)(s_x + (dx * 32 + cg * 8 + e) * CIP + row * XPP + oct * 8) = w[e];
      }
    }
    __syncthreads();
#pragma unroll
    for (int st = 0; st < NP / 32; ++st) {
      const int pk = st * 32 + (lane >> 4) * 8;  // first of this lane's 8 pixels (same tile row)
      const int prow = pk / TW, pcol = pk % TW;
      const bf16x8_t afr = *(const bf16x8_t*)(s_dp + (mt * 16 + (lane & 15)) * DPP + pk);
#pragma unroll
      for (int tap = 0; tap < TAPS; ++tap) {
        const int dy = TAPS == 9 ? tap / 3 : 0, dx = TAPS == 9 ? tap % 3 : 0;
        const bf16x8_t bfr =
            *(const bf16x8_t*)(s_x + (dx * 32 + nt * 16 + (lane & 15)) * CIP + (prow + dy) * XPP + pcol);
        acc[tap] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bfr, acc[tap], 0, 0, 0);
      }
    }
  }
  // lane holds dW[co = co0 + mt*16 + 4*(lane>>4) + j][ci = ci0 + nt*16 + (lane&15)] per tap
  const int ci = ci0 + nt * 16 + (lane & 15);
  float* ps = part + (int64_t)split * g.cout * g.cin * TAPS;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int co = co0 + mt * 16 + 4 * (lane >> 4) + j;
    if (co >= g.cout || ci >= g.cin) continue;
#pragma unroll
    for (int tap = 0; tap < TAPS; ++tap) ps[((int64_t)co * g.cin + ci) * TAPS + tap] = acc[tap][j];
  }
}

// Weight gradient of a 1x1 layer, dW[co][ci] = sum over pixels p of
// dPre[p][co] * X[p][ci], on MFMA 16x16x32 BF16 with A = dPre^T (M = output
// channels, K = pixels) and B = X (N = input channels). A workgroup owns a
// 128 x 128 (co, ci) tile, so every pixel's data is read once per tile; wave
// w computes the 64 x 64 quarter (w / 2, w % 2) as 4 x 4 MFMA tiles. The
// pixels are taken in stages of 64 (within one sample), stages z, z + nsplit,
// ... for split z. Per stage, thread t < 128 loads an 8-pixel x 8-channel
// block of dPre and thread t >= 128 one of X (coalesced 16-byte loads along
// the channels), transposes it in registers and writes it to LDS as 16-byte
// rows [channel][8 pixels]; the next stage's loads are issued before the
// current stage's MFMA loop. The partial sums are written in the layout
// [co][ci < cin] of the split's row; k_reduce_rows sums the splits in a
// fixed order.
constexpr int kW1T = 128;          // output and input channels per workgroup
constexpr int kW1P = 64;           // pixels per stage
constexpr int kW1PP = kW1P + 8;    // LDS pitch (bf16) of a channel row

__global__ __launch_bounds__(256) void k_wgrad1(WgradGeo g, const bf16_t* __restrict__ dp,
                                                const bf16_t* __restrict__ x, float* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) bf16_t s_dp[kW1T * kW1PP];
  __shared__ __attribute__((aligned(16))) bf16_t s_x[kW1T * kW1PP];
  const int co0 = blockIdx.x * kW1T, ci0 = blockIdx.y * kW1T;
  const int split = blockIdx.z, nsplit = gridDim.z;
  const int npix = g.H * g.W;
  const int sps = (npix + kW1P - 1) / kW1P;  // stages per sample
  const int stages = sps * g.nb;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  // staging role: operand (0 = dPre, 1 = X), channel group and pixel octet
  const int which = t >> 7, oct = t & 7, cg = (t >> 3) & 15;
  const int ch = (which ? ci0 : co0) + cg * 8;
  const bool ch_ok = which ? ch < g.cin8 : ch < g.cout;
  const int pitch = which ? g.cin8 : g.dp_pitch;
  const bf16_t* src = which ? x : dp;
  const int64_t bstride = which ? g.x_bstride : g.dp_bstride;
  bf16_t* dst = (which ? s_x : s_dp) + (cg * 8) * kW1PP + oct * 8;

  f32x4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  uint4 v[8];
  auto issue = [&](int st) {
    const int smp = st / sps, p0 = (st - smp * sps) * kW1P + oct * 8;
    const bf16_t* b = src + smp * bstride + ch;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      v[r] = make_uint4(0, 0, 0, 0);
      if (ch_ok && p0 + r < npix) v[r] = *(const uint4*)(b + (int64_t)(p0 + r) * pitch);
    }
  };
  if (split < stages) issue(split);
  for (int st = split; st < stages; st += nsplit) {
    __syncthreads();  // the previous stage's MFMA loop is done with LDS
    {
      uint4 w[8];
      transpose8x8_bf16(v, w);
#pragma unroll
      for (int e = 0; e < 8; ++e) *(uint4*)(dst + e * kW1PP) = w[e];
    }
    __syncthreads();
    if (st + nsplit < stages) issue(st + nsplit);
#pragma unroll
    for (int ks = 0; ks < kW1P / 32; ++ks) {
      const int k = ks * 32 + (lane >> 4) * 8;
      bf16x8_t af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = *(const bf16x8_t*)(s_dp + (wm * 64 + i * 16 + (lane & 15)) * kW1PP + k);
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = *(const bf16x8_t*)(s_x + (wn * 64 + j * 16 + (lane & 15)) * kW1PP + k);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  }
  // lane holds dW[co0 + 64 wm + 16 i + 4 (lane >> 4) + q][ci0 + 64 wn + 16 j + (lane & 15)]
  float* ps = part + (int64_t)split * g.cout * g.cin;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int ci = ci0 + wn * 64 + j * 16 + (lane & 15);
    if (ci >= g.cin) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int co = co0 + wm * 64 + i * 16 + 4 * (lane >> 4) + q;
        if (co < g.cout) ps[(int64_t)co * g.cin + ci] = acc[i][j][q];
      }
  }
}

// out[k] = scale * sum_b part[b][k] (fixed order, FP64 accumulation). A
// workgroup handles 32 consecutive k; its 8 thread groups sum the rows
// g, g + 8, ... and the 8 group sums are added in order.
__global__ __launch_bounds__(256) void k_reduce_rows(const float* __restrict__ part, int nparts, int64_t len,
                                                     float scale, float* __restrict__ out) {
  __shared__ double red[8][32];
  const int kk = threadIdx.x & 31, g = threadIdx.x >> 5;
  const int64_t k = (int64_t)blockIdx.x * 32 + kk;
  // rows g, g + 8, ... in four interleaved partial sums (their loads in
  // flight together), added in a fixed order
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (k < len) {
    int b = g;
    for (; b + 24 < nparts; b += 32) {
      s0 += part[(int64_t)b * len + k];
      s1 += part[(int64_t)(b + 8) * len + k];
      s2 += part[(int64_t)(b + 16) * len + k];
      s3 += part[(int64_t)(b + 24) * len + k];
    }
    for (; b < nparts; b += 8) s0 += part[(int64_t)b * len + k];
  }
  const double s = (s0 + s1) + (s2 + s3);
  red[g][kk] = s;
  __syncthreads();
  if (g == 0 && k < len) {
    double tot = 0.0;
    for (int q = 0; q < 8; ++q) tot += red[q][kk];
    out[k] = (float)(scale * tot);
  }
}

// Bias gradient partials: part[b][c] = sum over workgroup b's pixels of d[p][c].
// Thread t reads 8 channels (c8 = t % (C/8)) of the pixels of phase t / (C/8);
// the phases are summed in LDS in a fixed order. Requires C % 8 == 0, C <= 2048.
__global__ __launch_bounds__(256) void k_bias_grad(const bf16_t* __restrict__ d, int64_t npix, int pitch, int off,
                                                   int C, float* __restrict__ part) {
  __shared__ float red[256 * 8];
  const int c8n = C / 8;
  const int G = 256 / c8n;  // pixel phases per workgroup
  const int t = threadIdx.x;
  const int c8 = t % c8n, g = t / c8n;
  float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (g < G) {
    // four pixels' loads in flight per thread
    const int64_t step = (int64_t)gridDim.x * G;
    for (int64_t p = (int64_t)blockIdx.x * G + g; p < npix; p += 4 * step) {
      uint4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t pu = p + u * step;
        v[u] = pu < npix ? *(const uint4*)(d + pu * pitch + off + c8 * 8) : make_uint4(0, 0, 0, 0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t w4[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          acc[2 * e] += bf2f((bf16_t)(w4[e] & 0xffff));
          acc[2 * e + 1] += bf2f((bf16_t)(w4[e] >> 16));
        }
      }
    }
  }
#pragma unroll
  for (int e = 0; e < 8; ++e) red[t * 8 + e] = acc[e];
  __syncthreads();
  for (int c = t; c < C; c += 256) {
    float sacc = 0.f;
    for (int gg = 0; gg < G; ++gg) sacc += red[(gg * c8n + c / 8) * 8 + (c % 8)];
    part[(int64_t)blockIdx.x * C + c] = sacc;
  }
}

// In-place activation backward: d *= relu'(out) (mode 1) or tanh'(out) (mode 2).
// Eight channels per thread (C, pitches and offsets are multiples of 8).
__global__ void k_act_bwd(bf16_t* __restrict__ d, int dpitch, const bf16_t* __restrict__ out, int opitch, int ooff,
                          int C, int64_t npix, int mode) {
  const int c8n = C / 8;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= npix * c8n) return;
  const int64_t p = idx / c8n;
  const int c = (int)(idx - p * c8n) * 8;
  uint4* dp = (uint4*)(d + p * dpitch + c);
  const uint4 dv = *dp, ov = *(const uint4*)(out + p * opitch + ooff + c);
  const uint32_t a[4] = {dv.x, dv.y, dv.z, dv.w}, b[4] = {ov.x, ov.y, ov.z, ov.w};
  uint32_t o[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    float lo = bf2f((bf16_t)(a[e] & 0xffff)), hi = bf2f((bf16_t)(a[e] >> 16));
    const float olo = bf2f((bf16_t)(b[e] & 0xffff)), ohi = bf2f((bf16_t)(b[e] >> 16));
    if (mode == 1) {
      lo = olo > 0.f ? lo : 0.f;
      hi = ohi > 0.f ? hi : 0.f;
    } else {
      lo *= 1.f - olo * olo;
      hi *= 1.f - ohi * ohi;
    }
    o[e] = (uint32_t)f2bf(lo) | ((uint32_t)f2bf(hi) << 16);
  }
  *dp = make_uint4(o[0], o[1], o[2], o[3]);
}

// dst[p][c] (+)= src[p][soff + c], c < C.
__global__ void k_copy_ch(const bf16_t* __restrict__ src, int spitch, int soff, bf16_t* __restrict__ dst, int dpitch,
                          int C, int64_t npix, int accumulate) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= npix * C) return;
  const int64_t p = idx / C;
  const int c = (int)(idx - p * C);
  float v = bf2f(src[p * spitch + soff + c]);
  if (accumulate) v += bf2f(dst[p * dpitch + c]);
  dst[p * dpitch + c] = f2bf(v);
}

// Backward of nearest 2x upsampling: coarse[p][c] = sum of the 4 fine pixels.
__global__ void k_up_bwd(int Hc, int Wc, int C, const bf16_t* __restrict__ fine, int fpitch, int64_t f_bs,
                         bf16_t* __restrict__ coarse, int64_t c_bs) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)Hc * Wc * C) return;
  const int c = (int)(idx % C);
  const int64_t p = idx / C;
  const int y = (int)(p / Wc), xx = (int)(p - (int64_t)y * Wc);
  const bf16_t* f = fine + blockIdx.y * f_bs;
  float s = 0.f;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) s += bf2f(f[((int64_t)(2 * y + a) * 2 * Wc + 2 * xx + b) * fpitch + c]);
  coarse[blockIdx.y * c_bs + p * C + c] = f2bf(s);
}

// Backward of 2x2 average pooling: dE[2y+a][2x+b][c] += 0.25 * dpool[y][x][c].
__global__ void k_pool_bwd(int Hc, int Wc, int C, const bf16_t* __restrict__ dpool, int ppitch, int64_t p_bs,
                           bf16_t* __restrict__ dE, int64_t e_bs) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)Hc * Wc * C) return;
  const int c = (int)(idx % C);
  const int64_t p = idx / C;
  const int y = (int)(p / Wc), xx = (int)(p - (int64_t)y * Wc);
  const float g = 0.25f * bf2f(dpool[blockIdx.y * p_bs + p * ppitch + c]);
  bf16_t* e = dE + blockIdx.y * e_bs;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      bf16_t* q = e + ((int64_t)(2 * y + a) * 2 * Wc + 2 * xx + b) * C + c;
      *q = f2bf(bf2f(*q) + g);
    }
}

// ---------------------------------------------------------------------------
// Per-sample Mesh-Conv local weights (each sample has its own grid): the
// level arrays of sample s start at lv + s * lv_stride. A workgroup computes
// the hidden layer of Phi for 32 pixels, then writes eta[p][c] with the
// channel index fastest across threads.
constexpr int kEtaMPix = 128;  // pixels per workgroup of k_eta_multi
__global__ __launch_bounds__(256) void k_eta_multi(int H, int W, int cin, int cin8, int hid,
                                                   const float* __restrict__ lv, int64_t lv_stride,
                                                   const float* __restrict__ W1, const float* __restrict__ b1,
                                                   const float* __restrict__ W2, const float* __restrict__ b2,
                                                   bf16_t* __restrict__ eta, int64_t e_bs) {
  // Phi's output layer in LDS, transposed ([hid][cin] then b2) so that lanes
  // of consecutive channels read consecutive words; kEtaMPix pixels per
  // workgroup in batches of 32
  extern __shared__ float s_w2[];
  __shared__ float s_h[32][33];
  float* s_b2 = s_w2 + hid * cin;
  for (int u = threadIdx.x; u < cin * hid; u += 256) s_w2[(u % hid) * cin + u / hid] = W2[u];
  for (int u = threadIdx.x; u < cin; u += 256) s_b2[u] = b2[u];
  const int64_t npix = (int64_t)H * W;
  const float* L = lv + blockIdx.y * lv_stride;
  bf16_t* out = eta + blockIdx.y * e_bs;
  for (int64_t p0 = (int64_t)blockIdx.x * kEtaMPix; p0 < min(npix, (int64_t)(blockIdx.x + 1) * kEtaMPix); p0 += 32) {
    __syncthreads();
    for (int u = threadIdx.x; u < 32 * hid; u += 256) {
      const int q = u / hid, a = u - q * hid;
      const int64_t p = min(p0 + q, npix - 1);
      const int j = (int)(p / W), i = (int)(p - (int64_t)j * W);
      const float d0 = L[i], d1 = L[W + i], d2 = L[3 * W + j], d3 = L[3 * W + H + j];
      s_h[q][a] = tanh_nn(b1[a] + W1[a * 4] * d0 + W1[a * 4 + 1] * d1 + W1[a * 4 + 2] * d2 + W1[a * 4 + 3] * d3);
    }
    __syncthreads();
    for (int u = threadIdx.x; u < 32 * cin8; u += 256) {
      const int q = u / cin8, c = u - q * cin8;
      const int64_t p = p0 + q;
      if (p >= npix) continue;
      float e = 0.f;
      if (c < cin) {
        float phi = s_b2[c];
        for (int a = 0; a < hid; ++a) phi += s_w2[a * cin + c] * s_h[q][a];
        e = exp_nn(-phi * phi);
      }
      out[p * cin8 + c] = f2bf(e);
    }
  }
}

// Mesh-Conv local-weight backward. Given dXbar (gradient of the weighted
// input) and the layer input X: dX = eta * dXbar (written in place of dXbar)
// and, through dEta = dXbar * X and eta = exp(-Phi^2), the gradients of Phi's
// parameters. A workgroup handles 32-pixel batches of a contiguous pixel
// range (npb <= 32 pixels per batch, as many as the LDS holds for this
// layer's width). In the channel phase thread t owns the channel slots t % ns + k ns
// (ns = min(cin8, 256), k < KS) and pixel phase t / ns, and issues the loads
// of 8 pixels before using them. In the hidden phase thread t < S (S = the largest
// multiple of hid up to 256) owns hidden unit t % hid and the pixels t / hid,
// t / hid + S / hid, ..., so it accumulates its unit's W1 and b1 gradients
// itself. At the end the per-thread sums are reduced in a fixed order and one
// partial row [W1 (hid*4) | b1 (hid) | W2 (cin*hid) | b2 (cin)] (the layout
// of these parameters in the flat vector) is written. HC = hid rounded up to
// a power of two; KS >= cin8 / 256 channel slots per thread.
constexpr int kEtaPix = 32;
constexpr int kEtaGrp = 8;  // pixels whose loads are in flight together
template <int HC, int KS>
__global__ __launch_bounds__(256) void k_eta_bwd(int H, int W, int cin, int cin8, int hid, int nb,
                                                 const float* __restrict__ lv, int64_t lv_stride,
                                                 const float* __restrict__ W1, const float* __restrict__ b1,
                                                 const float* __restrict__ W2, const float* __restrict__ b2,
                                                 const bf16_t* __restrict__ x, const bf16_t* __restrict__ eta,
                                                 int64_t e_bs, bf16_t* __restrict__ dxb, float* __restrict__ part,
                                                 int npb) {
  extern __shared__ float sm[];
  const int cinp = cin + 1;                 // odd row pitch: rows start in different banks
  float* s_h = sm;                          // [kEtaPix][HC] hidden activations
  float* s_d = s_h + kEtaPix * HC;          // [kEtaPix][4] distances
  float* s_w2 = s_d + kEtaPix * 4;          // [hid][cinp] (transposed)
  float* s_dphi = s_w2 + cinp * hid;        // [npb][cinp]; reused for the final reductions
  __shared__ int s_smp[kEtaPix], s_pix[kEtaPix];  // sample and pixel of each batch pixel
  const int64_t npix = (int64_t)H * W, ntot = npix * nb;
  const int npix32 = H * W;
  const int64_t per = (ntot + gridDim.x - 1) / gridDim.x;
  const int64_t pbeg = blockIdx.x * per, pend = min(ntot, pbeg + per);
  const int t = threadIdx.x;
  const int ns = cin8 < 256 ? cin8 : 256;
  const int phases = 256 / ns;
  const int slot = t % ns, ph = t / ns;
  const bool active = ph < phases;
  const int qstep = 256 / hid, S = qstep * hid;
  const int my_a = t % hid, my_q = t / hid;  // hidden phase (t < S)
  for (int u = t; u < cin * hid; u += 256) s_w2[(u % hid) * cinp + u / hid] = W2[u];
  // the thread's own channels' row of Phi's output layer in registers when it
  // is small enough (else read from LDS)
  constexpr bool W2REG = KS * HC <= 32;
  float aw2[KS][HC], ab2[KS], b2r[KS], w2r[W2REG ? KS : 1][W2REG ? HC : 1];
  float aw1[5] = {0.f, 0.f, 0.f, 0.f, 0.f};  // W1 row and b1 of unit my_a
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    const int c = slot + ns * k;
    ab2[k] = 0.f;
    b2r[k] = c < cin ? b2[c] : 0.f;
#pragma unroll
    for (int q = 0; q < HC; ++q) {
      aw2[k][q] = 0.f;
      if (W2REG) w2r[W2REG ? k : 0][W2REG ? q : 0] = (c < cin && q < hid) ? W2[c * hid + q] : 0.f;
    }
  }
  for (int64_t p0 = pbeg; p0 < pend; p0 += npb) {
    const int np = (int)min((int64_t)npb, pend - p0);
    __syncthreads();
    for (int u = t; u < np * hid; u += 256) {
      const int q = u / hid, a = u - q * hid;
      const int gp = (int)(p0 + q);  // the host keeps npix * nb below 2^31
      const int smp = gp / npix32;
      const int p = gp - smp * npix32;
      const int j = p / W, i = p - j * W;
      const float* L = lv + smp * lv_stride;
      const float d0 = L[i], d1 = L[W + i], d2 = L[3 * W + j], d3 = L[3 * W + H + j];
      s_h[q * HC + a] = tanh_nn(b1[a] + W1[a * 4] * d0 + W1[a * 4 + 1] * d1 + W1[a * 4 + 2] * d2 + W1[a * 4 + 3] * d3);
      if (a == 0) {
        s_d[q * 4] = d0;
        s_d[q * 4 + 1] = d1;
        s_d[q * 4 + 2] = d2;
        s_d[q * 4 + 3] = d3;
        s_smp[q] = smp;
        s_pix[q] = p;
      }
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const int c = slot + ns * k;
        if (c >= cin8) continue;
        for (int qb = ph; qb < np; qb += phases * kEtaGrp) {
          float gv[kEtaGrp], xv[kEtaGrp], ev[kEtaGrp];
          int64_t ov[kEtaGrp];
#pragma unroll
          for (int e = 0; e < kEtaGrp; ++e) {
            const int q = qb + phases * e;
            gv[e] = xv[e] = ev[e] = 0.f;
            ov[e] = -1;
            if (q < np) {
              ov[e] = (p0 + q) * cin8 + c;
              gv[e] = bf2f(dxb[ov[e]]);
              xv[e] = bf2f(x[ov[e]]);
              ev[e] = bf2f(eta[s_smp[q] * e_bs + (int64_t)s_pix[q] * cin8 + c]);
            }
          }
#pragma unroll
          for (int e = 0; e < kEtaGrp; ++e) {
            const int q = qb + phases * e;
            if (ov[e] < 0) continue;
            dxb[ov[e]] = f2bf(ev[e] * gv[e]);
            if (c >= cin) continue;
            float phi = b2r[k];
#pragma unroll
            for (int a = 0; a < HC; ++a)
              if (a < hid)
                phi += (W2REG ? w2r[W2REG ? k : 0][W2REG ? a : 0] : s_w2[a * cinp + c]) * s_h[q * HC + a];
            const float ef = exp_nn(-phi * phi);
            const float dphi = gv[e] * xv[e] * (-2.f * phi * ef);
            s_dphi[q * cinp + c] = dphi;
            ab2[k] += dphi;
#pragma unroll
            for (int a = 0; a < HC; ++a)
              if (a < hid) aw2[k][a] += dphi * s_h[q * HC + a];
          }
        }
      }
    }
    __syncthreads();
    // dz[q][a] = (sum_c W2[c][a] dphi[q][c]) (1 - h^2); the unit's W1 / b1 sums
    if (t < S) {
      const float* w = s_w2 + my_a * cinp;
      for (int q = my_q; q < np; q += qstep) {
        const float* f = s_dphi + q * cinp;
        float e0 = 0.f, e1 = 0.f, e2 = 0.f, e3 = 0.f;
        int c = 0;
        for (; c + 4 <= cin; c += 4) {
          e0 += w[c] * f[c];
          e1 += w[c + 1] * f[c + 1];
          e2 += w[c + 2] * f[c + 2];
          e3 += w[c + 3] * f[c + 3];
        }
        for (; c < cin; ++c) e0 += w[c] * f[c];
        const float h = s_h[q * HC + my_a];
        const float dz = ((e0 + e1) + (e2 + e3)) * (1.f - h * h);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) aw1[kk] += dz * s_d[q * 4 + kk];
        aw1[4] += dz;
      }
    }
  }
  const int len = hid * 5 + cin * hid + cin;
  float* row = part + (int64_t)blockIdx.x * len;
  float* red = s_dphi;  // >= 256 * (HC + 1) floats
  // W1 / b1: the threads of one unit, in order of their pixel offset
  __syncthreads();
#pragma unroll
  for (int kk = 0; kk < 5; ++kk) red[t * 5 + kk] = t < S ? aw1[kk] : 0.f;
  __syncthreads();
  if (t < hid * 5) {
    const int a = t / 5, kk = t - a * 5;
    float acc = 0.f;
    for (int q = 0; q < qstep; ++q) acc += red[(q * hid + a) * 5 + kk];
    if (kk < 4) row[a * 4 + kk] = acc;
    else row[hid * 4 + a] = acc;
  }
  // W2 / b2: the per-phase sums of each channel
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    __syncthreads();
#pragma unroll
    for (int a = 0; a <= HC; ++a)
      if (a <= hid) red[t * (HC + 1) + a] = a < hid ? aw2[k][a < HC ? a : 0] : ab2[k];
    __syncthreads();
    for (int u = t; u < ns * (hid + 1); u += 256) {
      const int sl = u / (hid + 1), a = u - sl * (hid + 1);
      const int c = sl + ns * k;
      if (c >= cin) continue;
      float acc = 0.f;
      for (int q = 0; q < phases; ++q) acc += red[(q * ns + sl) * (HC + 1) + a];
      if (a < hid) row[hid * 5 + c * hid + a] = acc;
      else row[hid * 5 + cin * hid + c] = acc;
    }
  }
}

// Static channels of the activation buffers of nb samples on their own grids.
__global__ void k_fill_static_multi(int H, int W, int pitch, int coff, const float* __restrict__ lv, int64_t lv_stride,
                                    const uint8_t* const* __restrict__ masks, int moff, bf16_t* __restrict__ buf,
                                    int64_t bstride) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)H * W) return;
  const int j = (int)(p / W), i = (int)(p - (int64_t)j * W);
  const float* L = lv + blockIdx.y * lv_stride;
  bf16_t* b = buf + blockIdx.y * bstride + p * pitch;
  if (coff >= 0) {
    b[coff] = f2bf(L[2 * W + i]);
    b[coff + 1] = f2bf(L[3 * W + 2 * H + j]);
  }
  if (moff >= 0) {
    const uint8_t* m = masks ? masks[blockIdx.y] : nullptr;
    b[moff] = f2bf(m ? (float)m[p] : 0.f);
  }
}

// Trunk input channels (normalised centre coordinates, padded to 8).
__global__ void k_trunk_input(int H, int W, const float* __restrict__ tin, int64_t t_stride, bf16_t* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)H * W) return;
  const int j = (int)(p / W), i = (int)(p - (int64_t)j * W);
  const float* tt = tin + blockIdx.y * t_stride;
  bf16_t* o = out + ((int64_t)blockIdx.y * H * W + p) * 8;
  o[0] = f2bf(tt[i]);
  o[1] = f2bf(tt[W + j]);
  for (int c = 2; c < 8; ++c) o[c] = 0;
}

// DeepONet contraction y = gamma * sum_k B_k T_k (FP32 sum of BF16 operands).
// 16 lanes per pixel, 8 basis terms per lane per pass (P % 8 == 0).
__device__ __forceinline__ float dot8(uint4 a, uint4 b) {
  const uint32_t x[4] = {a.x, a.y, a.z, a.w}, y[4] = {b.x, b.y, b.z, b.w};
  float s = 0.f;
#pragma unroll
  for (int e = 0; e < 4; ++e)
    s += bf2f((bf16_t)(x[e] & 0xffff)) * bf2f((bf16_t)(y[e] & 0xffff)) +
         bf2f((bf16_t)(x[e] >> 16)) * bf2f((bf16_t)(y[e] >> 16));
  return s;
}

__device__ __forceinline__ float sum16(float v) {
#pragma unroll
  for (int o = 8; o >= 1; o >>= 1) v += __shfl_xor(v, o, 16);
  return v;
}

__global__ __launch_bounds__(256) void k_don_fwd(int64_t n, int P, const bf16_t* __restrict__ B,
                                                 const bf16_t* __restrict__ T, const float* __restrict__ gamma,
                                                 float* __restrict__ y) {
  const int64_t p = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
  const int l = threadIdx.x & 15;
  float s = 0.f;
  if (p < n)
    for (int k = l * 8; k < P; k += 128) s += dot8(*(const uint4*)(B + p * P + k), *(const uint4*)(T + p * P + k));
  s = sum16(s);
  if (p < n && l == 0) y[p] = gamma[0] * s;
}

__device__ __forceinline__ uint4 scale8(uint4 a, float c) {
  const uint32_t x[4] = {a.x, a.y, a.z, a.w};
  uint32_t o[4];
#pragma unroll
  for (int e = 0; e < 4; ++e)
    o[e] = (uint32_t)f2bf(c * bf2f((bf16_t)(x[e] & 0xffff))) | ((uint32_t)f2bf(c * bf2f((bf16_t)(x[e] >> 16))) << 16);
  return make_uint4(o[0], o[1], o[2], o[3]);
}

// Its backward for dy = scale * g: dB = gamma dy T, dT = gamma dy B, and
// per-workgroup partials of dgamma = sum dy sum_k B_k T_k.
__global__ __launch_bounds__(256) void k_don_bwd(int64_t n, int P, const bf16_t* __restrict__ B,
                                                 const bf16_t* __restrict__ T, const float* __restrict__ gamma,
                                                 const float* __restrict__ g, float scale, bf16_t* __restrict__ dB,
                                                 bf16_t* __restrict__ dT, float* __restrict__ part) {
  __shared__ double lds[kWaves];
  const int l = threadIdx.x & 15;
  const float gam = gamma[0];
  double acc = 0.0;
  // four pixels per pass, their loads issued together; 16 lanes per pixel,
  // lane l holding basis terms 8l .. 8l+7 (P <= 128: at most one group)
  const int k = l * 8;
  const bool kin = k < P;
  const int64_t step = (int64_t)gridDim.x * 16;
  for (int64_t p0 = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4); p0 < n; p0 += 4 * step) {
    uint4 b[4], t[4];
    float dy[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t p = p0 + u * step;
      const bool ok = p < n && kin;
      b[u] = ok ? *(const uint4*)(B + p * P + k) : make_uint4(0, 0, 0, 0);
      t[u] = ok ? *(const uint4*)(T + p * P + k) : make_uint4(0, 0, 0, 0);
      dy[u] = p < n ? scale * g[p] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t p = p0 + u * step;
      const float tot = sum16(dot8(b[u], t[u]));  // all 16 lanes of the pixel take part
      if (p < n) {
        const float gd = gam * dy[u];
        if (kin) {
          *(uint4*)(dB + p * P + k) = scale8(t[u], gd);
          *(uint4*)(dT + p * P + k) = scale8(b[u], gd);
        }
        if (l == 0) acc += (double)dy[u] * (double)tot;
      }
    }
  }
  acc = block_sum(acc, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = (float)acc;
}

// Residual loss pieces: res = R - Ay (stored), per-workgroup partials of res^2.
__global__ __launch_bounds__(256) void k_loss(int64_t n, const float* __restrict__ R, const float* __restrict__ Ay,
                                              float* __restrict__ res, double* __restrict__ part) {
  __shared__ double lds[kWaves];
  double acc = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
    const float v = R[p] - Ay[p];
    res[p] = v;
    acc += (double)v * v;
  }
  acc = block_sum(acc, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Supervised loss pieces, per sample s (blockIdx.y): partial sums of y, e,
// y^2, y e and e^2 ([nb][5][gridDim.x]).
__global__ __launch_bounds__(256) void k_sup_sums(int64_t N, const float* __restrict__ y,
                                                  const double* __restrict__ e, double* __restrict__ part) {
  __shared__ double lds[kWaves];
  const int s = blockIdx.y;
  const float* ys = y + (size_t)s * N;
  const double* es = e + (size_t)s * N;
  double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < N; p += (int64_t)gridDim.x * 256) {
    const double yv = ys[p], ev = es[p];
    a[0] += yv;
    a[1] += ev;
    a[2] += yv * yv;
    a[3] += yv * ev;
    a[4] += ev * ev;
  }
  for (int m = 0; m < 5; ++m) {
    const double v = block_sum(a[m], lds);
    if (threadIdx.x == 0) part[((size_t)s * 5 + m) * gridDim.x + blockIdx.x] = v;
  }
}

// Supervised loss L_s = 1 - a^2 / (b c) with a = y0.e0, b = |y0|^2, c = |e0|^2
// (centred fields) and its gradient, averaged over the nb samples:
// dL/dy = 2 a / (b c nb) (a/b y0 - e0) (zero mean, so the centring needs no
// further projection). A constant y (b = 0) or target (c = 0) gives L = 1
// and no gradient. Every workgroup reduces the partials in the same order.
__global__ __launch_bounds__(256) void k_sup_grad(int64_t N, int nb, const float* __restrict__ y,
                                                  const double* __restrict__ e, const double* __restrict__ part,
                                                  int nparts, float* __restrict__ dy, double* __restrict__ lsamp) {
  __shared__ double lds[kWaves];
  const int s = blockIdx.y;
  double S[5];
  for (int m = 0; m < 5; ++m) S[m] = reduce_partials(part + ((size_t)s * 5 + m) * nparts, nparts, lds);
  const double n = (double)N;
  const double my = S[0] / n, me = S[1] / n;
  const double a = S[3] - n * my * me;
  const double b = S[2] - n * my * my;
  const double c = S[4] - n * me * me;
  const bool ok = b > 0.0 && c > 0.0 && isfinite(a);
  const double L = ok ? 1.0 - a * a / (b * c) : 1.0;
  const double g = ok ? 2.0 * a / (b * c * (double)nb) : 0.0;
  const double ab = ok ? a / b : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) lsamp[s] = L;
  const float* ys = y + (size_t)s * N;
  const double* es = e + (size_t)s * N;
  float* ds = dy + (size_t)s * N;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < N; p += (int64_t)gridDim.x * 256)
    ds[p] = (float)(g * (ab * ((double)ys[p] - my) - (es[p] - me)));
}

// Per-sample partial sums of the A-norm loss: R.y, y.Ay, R.e (FP64).
__global__ __launch_bounds__(256) void k_anorm_sums(int64_t N, const float* __restrict__ y,
                                                    const float* __restrict__ Ay, const float* __restrict__ R,
                                                    const double* __restrict__ e, double* __restrict__ part) {
  __shared__ double lds[kWaves];
  const int s = blockIdx.y;
  const size_t o = (size_t)s * N;
  double a[3] = {0.0, 0.0, 0.0};
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < N; p += (int64_t)gridDim.x * 256) {
    const double yv = y[o + p], rv = R[o + p];
    a[0] += rv * yv;
    a[1] += yv * (double)Ay[o + p];
    a[2] += rv * e[o + p];
  }
  for (int m = 0; m < 3; ++m) {
    const double v = block_sum(a[m], lds);
    if (threadIdx.x == 0) part[((size_t)s * 3 + m) * gridDim.x + blockIdx.x] = v;
  }
}

// A-norm loss L_s = 1 - a^2 / (b c) with a = R.y, b = y.Ay, c = R.e, and its
// gradient averaged over the nb samples (A symmetric):
// dL/dy = (2 a / (b c nb)) (a/b A y - R). b <= 0 or c <= 0 gives L = 1 and no
// gradient. Every workgroup reduces the partials in the same order.
__global__ __launch_bounds__(256) void k_anorm_grad(int64_t N, int nb, const float* __restrict__ Ay,
                                                    const float* __restrict__ R, const double* __restrict__ part,
                                                    int nparts, float* __restrict__ dy, double* __restrict__ lsamp) {
  __shared__ double lds[kWaves];
  const int s = blockIdx.y;
  double S[3];
  for (int m = 0; m < 3; ++m) S[m] = reduce_partials(part + ((size_t)s * 3 + m) * nparts, nparts, lds);
  const double a = S[0], b = S[1], c = S[2];
  const bool ok = b > 0.0 && c > 0.0 && isfinite(a);
  const double L = ok ? 1.0 - a * a / (b * c) : 1.0;
  const double g = ok ? 2.0 * a / (b * c * (double)nb) : 0.0;
  const double ab = ok ? a / b : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) lsamp[s] = L;
  const size_t o = (size_t)s * N;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < N; p += (int64_t)gridDim.x * 256)
    dy[o + p] = (float)(g * (ab * (double)Ay[o + p] - (double)R[o + p]));
}

__global__ void k_sum_parts(const double* __restrict__ part, int n, double scale, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int k = 0; k < n; ++k) s += part[k];
  out[0] = scale * s;
}

// Adam (Kingma & Ba 2015, Alg. 1) on the FP32 master parameters. With
// clip > 0 the gradient is first scaled by min(1, clip / ||g||), ||g||^2 being
// the fixed-order sum of the kRedBlocks partial sums in gpart (the same bits
// in every workgroup).
__global__ __launch_bounds__(256) void k_adam(int64_t n, float* __restrict__ w, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                              float b2, float eps, float c1, float c2, const double* __restrict__ gpart,
                                              float clip) {
  __shared__ double lds[kWaves];
  float scale = 1.f;
  if (clip > 0.f) {
    const double gn = sqrt(reduce_partials(gpart, kRedBlocks, lds));
    if (gn > (double)clip) scale = (float)((double)clip / gn);
  }
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gk = g[k] * scale;
  const float mk = b1 * m[k] + (1.f - b1) * gk;
  const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  w[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// Sharpness-aware perturbation (Foret et al., 2021): w += rho g / |g|, with
// |g|^2 from the kRedBlocks partials of k_sumsq reduced in the same order by
// every workgroup; no change when g = 0.
__global__ __launch_bounds__(256) void k_sam_perturb(int64_t n, float* w, const float* g, const double* gpart,
                                                     float rho) {
  __shared__ double lds[kWaves];
  const double gn = sqrt(reduce_partials(gpart, kRedBlocks, lds));
  const float scale = gn > 0.0 ? (float)((double)rho / gn) : 0.f;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) w[k] += scale * g[k];
}

// ---------------------------------------------------------------------------
static unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

void launch_wgrad(int taps, const WgradGeo& g, const bf16_t* dp, const bf16_t* x, const bf16_t* eta, float* part,
                  int nsplit, hipStream_t s) {
  if (taps == 1 && !eta) {
    const dim3 grid1((g.cout + kW1T - 1) / kW1T, (g.cin8 + kW1T - 1) / kW1T, nsplit);
    k_wgrad1<<<grid1, 256, 0, s>>>(g, dp, x, part);
    return;
  }
  const dim3 grid((g.cout + 31) / 32, (g.cin8 + 31) / 32, nsplit);
  if (taps == 9) k_wgrad<9><<<grid, 256, 0, s>>>(g, dp, x, eta, part);
  else k_wgrad<1><<<grid, 256, 0, s>>>(g, dp, x, eta, part);
}

void launch_reduce_rows(const float* part, int nparts, int64_t len, float scale, float* out, hipStream_t s) {
  k_reduce_rows<<<(unsigned)((len + 31) / 32), 256, 0, s>>>(part, nparts, len, scale, out);
}

void launch_bias_grad(const bf16_t* d, int64_t npix, int pitch, int off, int C, float* part, int nparts,
                      hipStream_t s) {
  k_bias_grad<<<nparts, 256, 0, s>>>(d, npix, pitch, off, C, part);
}

void launch_act_bwd(bf16_t* d, int dpitch, const bf16_t* out, int opitch, int ooff, int C, int64_t npix, int mode,
                    hipStream_t s) {
  k_act_bwd<<<nblk(npix * (C / 8)), 256, 0, s>>>(d, dpitch, out, opitch, ooff, C, npix, mode);
}

void launch_copy_ch(const bf16_t* src, int spitch, int soff, bf16_t* dst, int dpitch, int C, int64_t npix, int acc,
                    hipStream_t s) {
  k_copy_ch<<<nblk(npix * C), 256, 0, s>>>(src, spitch, soff, dst, dpitch, C, npix, acc);
}

void launch_up_bwd(int Hc, int Wc, int C, const bf16_t* fine, int fpitch, int64_t f_bs, bf16_t* coarse, int64_t c_bs,
                   int nb, hipStream_t s) {
  k_up_bwd<<<dim3(nblk((int64_t)Hc * Wc * C), nb), 256, 0, s>>>(Hc, Wc, C, fine, fpitch, f_bs, coarse, c_bs);
}

void launch_pool_bwd(int Hc, int Wc, int C, const bf16_t* dpool, int ppitch, int64_t p_bs, bf16_t* dE, int64_t e_bs,
                     int nb, hipStream_t s) {
  k_pool_bwd<<<dim3(nblk((int64_t)Hc * Wc * C), nb), 256, 0, s>>>(Hc, Wc, C, dpool, ppitch, p_bs, dE, e_bs);
}

void launch_eta_multi(int H, int W, int cin, int cin8, int hid, const float* lv, int64_t lv_stride, const float* W1,
                      const float* b1, const float* W2, const float* b2, bf16_t* eta, int64_t e_bs, int nb,
                      hipStream_t s) {
  const size_t shm = sizeof(float) * ((size_t)hid * cin + cin);
  k_eta_multi<<<dim3((unsigned)(((int64_t)H * W + kEtaMPix - 1) / kEtaMPix), nb), 256, shm, s>>>(
      H, W, cin, cin8, hid, lv, lv_stride, W1, b1, W2, b2, eta, e_bs);
}

int eta_bwd_len(int cin, int hid) { return hid * 5 + cin * hid + cin; }

// LDS of one workgroup of k_eta_bwd, in floats, apart from the dphi rows.
static int64_t eta_bwd_fixed(int cin, int hid, int hc) { return (int64_t)kEtaPix * hc + kEtaPix * 4 + (int64_t)(cin + 1) * hid; }

// LDS available to one workgroup's dynamic allocation: the default 64 KiB
// limit less 1 KiB for the kernel's static arrays.
static int64_t lds_per_block() { return 63 * 1024; }

static int eta_bwd_hc(int hid) { return hid <= 4 ? 4 : hid <= 8 ? 8 : hid <= 16 ? 16 : 32; }

// Pixels per batch that fit the LDS (0: the layer is too wide).
static int eta_bwd_npb(int cin, int hid) {
  const int hc = eta_bwd_hc(hid);
  const int64_t room = lds_per_block() / (int64_t)sizeof(float) - eta_bwd_fixed(cin, hid, hc);
  if (room < 256 * (int64_t)(hc + 1)) return 0;  // the final reductions need this much
  return (int)std::min<int64_t>(kEtaPix, room / (cin + 1));
}

bool eta_bwd_fits(int cin, int cin8, int hid) { return cin8 <= 1024 && eta_bwd_npb(cin, hid) >= 1; }

void launch_eta_bwd(int H, int W, int cin, int cin8, int hid, int nb, const float* lv, int64_t lv_stride,
                    const float* W1, const float* b1, const float* W2, const float* b2, const bf16_t* x,
                    const bf16_t* eta, int64_t e_bs, bf16_t* dxb, float* part, int nparts, hipStream_t s) {
  const int hc = eta_bwd_hc(hid);
  const int npb = eta_bwd_npb(cin, hid);  // >= 1: the caller checked eta_bwd_fits
  const size_t shm = sizeof(float) * (eta_bwd_fixed(cin, hid, hc) +
                                      std::max<int64_t>((int64_t)npb * (cin + 1), 256 * (int64_t)(hc + 1)));
#define PPE_ETA_BWD(HC, KS)                                                                                    \
  k_eta_bwd<HC, KS><<<nparts, 256, shm, s>>>(H, W, cin, cin8, hid, nb, lv, lv_stride, W1, b1, W2, b2, x, eta, \
                                             e_bs, dxb, part, npb)
#define PPE_ETA_BWD_HC(KS)                  \
  if (hc == 4) PPE_ETA_BWD(4, KS);          \
  else if (hc == 8) PPE_ETA_BWD(8, KS);     \
  else if (hc == 16) PPE_ETA_BWD(16, KS);   \
  else PPE_ETA_BWD(32, KS)
  // channel slots per thread: cin8 <= 256 needs one, <= 512 two, <= 1024 four
  if (cin8 <= 256) { PPE_ETA_BWD_HC(1); }
  else if (cin8 <= 512) { PPE_ETA_BWD_HC(2); }
  else { PPE_ETA_BWD_HC(4); }
#undef PPE_ETA_BWD_HC
#undef PPE_ETA_BWD
}

void launch_fill_static_multi(int H, int W, int pitch, int coff, const float* lv, int64_t lv_stride,
                              const uint8_t* const* masks, int moff, bf16_t* buf, int64_t bstride, int nb,
                              hipStream_t s) {
  k_fill_static_multi<<<dim3(nblk((int64_t)H * W), nb), 256, 0, s>>>(H, W, pitch, coff, lv, lv_stride, masks, moff,
                                                                      buf, bstride);
}

void launch_trunk_input(int H, int W, const float* tin, int64_t t_stride, bf16_t* out, int nb, hipStream_t s) {
  k_trunk_input<<<dim3(nblk((int64_t)H * W), nb), 256, 0, s>>>(H, W, tin, t_stride, out);
}

void launch_don_fwd(int64_t n, int P, const bf16_t* B, const bf16_t* T, const float* gamma, float* y, hipStream_t s) {
  k_don_fwd<<<(unsigned)((n + 15) / 16), 256, 0, s>>>(n, P, B, T, gamma, y);
}

void launch_don_bwd(int64_t n, int P, const bf16_t* B, const bf16_t* T, const float* gamma, const float* g,
                    float scale, bf16_t* dB, bf16_t* dT, float* part, int nparts, hipStream_t s) {
  k_don_bwd<<<nparts, 256, 0, s>>>(n, P, B, T, gamma, g, scale, dB, dT, part);
}

void launch_loss(int64_t n, const float* R, const float* Ay, float* res, double* part, int nparts, hipStream_t s) {
  k_loss<<<nparts, 256, 0, s>>>(n, R, Ay, res, part);
}

void launch_sup_loss(int64_t N, int nb, const float* y, const double* e, double* part, int nparts, float* dy,
                     double* lsamp, hipStream_t s) {
  k_sup_sums<<<dim3(nparts, nb), 256, 0, s>>>(N, y, e, part);
  k_sup_grad<<<dim3(nparts, nb), 256, 0, s>>>(N, nb, y, e, part, nparts, dy, lsamp);
}

void launch_anorm_loss(int64_t N, int nb, const float* y, const float* Ay, const float* R, const double* e,
                       double* part, int nparts, float* dy, double* lsamp, hipStream_t s) {
  k_anorm_sums<<<dim3(nparts, nb), 256, 0, s>>>(N, y, Ay, R, e, part);
  k_anorm_grad<<<dim3(nparts, nb), 256, 0, s>>>(N, nb, Ay, R, part, nparts, dy, lsamp);
}

// Mesh-Conv local-weight backward with one local weight per node (Eqs.
// 17-18 as written: Phi has one output). Given dXbar (gradient of the
// weighted input) and the layer input X: dX = eta * dXbar (in place of
// dXbar), dEta[p] = sum_c dXbar[p][c] X[p][c], and through eta = exp(-Phi^2),
// Phi = W2 . tanh(W1 d + b1) + b2 (d the node's four distances), the
// gradients of Phi's parameters. One thread per pixel of the batch
// (grid-stride). Each thread sums its pixels' parameter gradients; a wave
// adds its lanes by a butterfly and the workgroup its waves in order, into
// one partial row [W1 (hid*4) | b1 (hid) | W2 (hid) | b2] (the layout of
// these parameters in the flat vector). HC = hid rounded up to a power of two.
template <int HC>
__global__ __launch_bounds__(256) void k_eta_bwd_node(int H, int W, int cin8, int hid, int nb,
                                                      const float* __restrict__ lv, int64_t lv_stride,
                                                      const float* __restrict__ W1, const float* __restrict__ b1,
                                                      const float* __restrict__ W2, const float* __restrict__ b2,
                                                      const bf16_t* __restrict__ x, const bf16_t* __restrict__ eta,
                                                      bf16_t* __restrict__ dxb, float* __restrict__ part) {
  constexpr int NV = HC * 6 + 1;  // accumulated values: W1 (4 HC), b1, W2, b2
  __shared__ float s_w[kWaves][NV];
  float acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.f;
  const int64_t npix = (int64_t)H * W, ntot = npix * nb;
  for (int64_t gp = (int64_t)blockIdx.x * 256 + threadIdx.x; gp < ntot; gp += (int64_t)gridDim.x * 256) {
    const int smp = (int)(gp / npix);
    const int p = (int)(gp - smp * npix);
    const int j = p / W, i = p - j * W;
    const float* L = lv + smp * lv_stride;
    const float d[4] = {L[i], L[W + i], L[3 * W + j], L[3 * W + H + j]};
    // dEta and dX over the pixel's channels (eta: one value per pixel of each sample)
    const float e = bf2f(eta[gp]);
    const uint4* xr = (const uint4*)(x + gp * cin8);
    uint4* gr = (uint4*)(dxb + gp * cin8);
    float se = 0.f;
    for (int c8 = 0; c8 < cin8 / 8; ++c8) {
      const uint4 gv = gr[c8], xv = xr[c8];
      const uint32_t ga[4] = {gv.x, gv.y, gv.z, gv.w}, xa[4] = {xv.x, xv.y, xv.z, xv.w};
      uint32_t o[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float g0 = bf2f((bf16_t)(ga[k] & 0xffff)), g1 = bf2f((bf16_t)(ga[k] >> 16));
        se += g0 * bf2f((bf16_t)(xa[k] & 0xffff)) + g1 * bf2f((bf16_t)(xa[k] >> 16));
        o[k] = (uint32_t)f2bf(e * g0) | ((uint32_t)f2bf(e * g1) << 16);
      }
      gr[c8] = make_uint4(o[0], o[1], o[2], o[3]);
    }
    // Phi and its parameters' gradients at this node
    float h[HC];
    float phi = b2[0];
#pragma unroll
    for (int a = 0; a < HC; ++a) {
      h[a] = 0.f;
      if (a < hid) {
        h[a] = tanh_nn(b1[a] + W1[a * 4] * d[0] + W1[a * 4 + 1] * d[1] + W1[a * 4 + 2] * d[2] + W1[a * 4 + 3] * d[3]);
        phi += W2[a] * h[a];
      }
    }
    const float dphi = se * (-2.f * phi * exp_nn(-phi * phi));
#pragma unroll
    for (int a = 0; a < HC; ++a) {
      if (a >= hid) continue;
      const float dz = dphi * W2[a] * (1.f - h[a] * h[a]);
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[a * 4 + k] += dz * d[k];
      acc[HC * 4 + a] += dz;
      acc[HC * 5 + a] += dphi * h[a];
    }
    acc[HC * 6] += dphi;
  }
  // lanes of a wave (butterfly), then the waves in order
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    float v = acc[k];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) s_w[wv][k] = v;
  }
  __syncthreads();
  const int len = hid * 6 + 1;
  float* row = part + (int64_t)blockIdx.x * len;
  for (int u = threadIdx.x; u < len; u += 256) {
    // u: W1 (a * 4 + k) | b1 (a) | W2 (a) | b2
    const int k = u < hid * 4 ? u : u < hid * 5 ? HC * 4 + (u - hid * 4) : u < hid * 6 ? HC * 5 + (u - hid * 5) : HC * 6;
    float t = 0.f;
    for (int w = 0; w < kWaves; ++w) t += s_w[w][k];
    row[u] = t;
  }
}

int eta_bwd_node_len(int hid) { return hid * 6 + 1; }

void launch_eta_bwd_node(int H, int W, int cin8, int hid, int nb, const float* lv, int64_t lv_stride,
                         const float* W1, const float* b1, const float* W2, const float* b2, const bf16_t* x,
                         const bf16_t* eta, bf16_t* dxb, float* part, int nparts, hipStream_t s) {
  if (hid <= 8)
    k_eta_bwd_node<8><<<nparts, 256, 0, s>>>(H, W, cin8, hid, nb, lv, lv_stride, W1, b1, W2, b2, x, eta, dxb, part);
  else if (hid <= 16)
    k_eta_bwd_node<16><<<nparts, 256, 0, s>>>(H, W, cin8, hid, nb, lv, lv_stride, W1, b1, W2, b2, x, eta, dxb, part);
  else
    k_eta_bwd_node<32><<<nparts, 256, 0, s>>>(H, W, cin8, hid, nb, lv, lv_stride, W1, b1, W2, b2, x, eta, dxb, part);
}

void launch_sum_parts(const double* part, int n, double scale, double* out, hipStream_t s) {
  k_sum_parts<<<1, 64, 0, s>>>(part, n, scale, out);
}

void launch_adam(int64_t n, float* w, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                 float c1, float c2, const double* gpart, float clip, hipStream_t s) {
  k_adam<<<nblk(n), 256, 0, s>>>(n, w, g, m, v, lr, b1, b2, eps, c1, c2, gpart, clip);
}

void launch_sam_perturb(int64_t n, float* w, const float* g, const double* gpart, float rho, hipStream_t s) {
  k_sam_perturb<<<nblk(n), 256, 0, s>>>(n, w, g, gpart, rho);
}

}  // namespace ppe
