// Tile geometry, buffer loads and the 5-point stencil on register tiles
// shared by the PCG kernels (HIP, gfx950).
#pragma once
#include "common.hpp"

namespace ppe {

template <typename T>
struct ColCtx {
  int i, ih;
  bool ok, hok;
  T hx, gw, ge;    // own column
  T hxh, gwh, geh; // halo column (lanes 0 and 63)
};

template <typename T>
__device__ __forceinline__ ColCtx<T> col_ctx(int nx, const T* hx, const T* gx, int i0) {
  ColCtx<T> c;
  const int lane = threadIdx.x & (kWave - 1);
  c.i = i0 + lane;
  c.ok = c.i < nx;
  c.ih = (lane == 0) ? c.i - 1 : c.i + 1;
  c.hok = (lane == 0 || lane == kWave - 1) && c.ih >= 0 && c.ih < nx;
  c.hx = c.ok ? hx[c.i] : T(0);
  c.gw = c.ok ? gx[c.i] : T(0);
  c.ge = c.ok ? gx[c.i + 1] : T(0);
  c.hxh = c.hok ? hx[c.ih] : T(0);
  c.gwh = c.hok ? gx[c.ih] : T(0);
  c.geh = c.hok ? gx[c.ih + 1] : T(0);
  return c;
}

template <typename T>
__device__ __forceinline__ T stencil5(T vc, T ve, T vw, T vn, T vs, T hyj, T gs, T gn, T hx, T gw,
                                      T ge) {
  return hyj * (ge * (vc - ve) + gw * (vc - vw)) + hx * (gn * (vc - vn) + gs * (vc - vs));
}

// East/west neighbours of every lane's value: lane i receives lanes i+1 and
// i-1 of the wavefront; lanes 63 and 0 take the halo value instead.
// FP32 uses DPP wave shifts (wave_shl:1 reads lane i+1, wave_shr:1 lane i-1);
// FP64 uses lane shuffles.
__device__ __forceinline__ void east_west(float vcur, float vh, float& ve, float& vw) {
  const int lane = threadIdx.x & (kWave - 1);
  const int bits = __float_as_int(vcur);
  const float e = __int_as_float(__builtin_amdgcn_update_dpp(0, bits, 0x130, 0xf, 0xf, false));
  const float w = __int_as_float(__builtin_amdgcn_update_dpp(0, bits, 0x138, 0xf, 0xf, false));
  ve = (lane == kWave - 1) ? vh : e;
  vw = (lane == 0) ? vh : w;
}

__device__ __forceinline__ void east_west(double vcur, double vh, double& ve, double& vw) {
  const int lane = threadIdx.x & (kWave - 1);
  const double e = __shfl_down(vcur, 1, kWave);
  const double w = __shfl_up(vcur, 1, kWave);
  ve = (lane == kWave - 1) ? vh : e;
  vw = (lane == 0) ? vh : w;
}

// Tile placement. A solve's workgroups form a 1D grid of 8 * ceil(T / 8)
// (T = tiles of 64 columns x 4R rows). Workgroups are dispatched round-robin
// over the 8 XCDs, so workgroup b runs on XCD b % 8; it takes logical tile
// (b % 8) * ceil(T / 8) + b / 8. Each XCD thus owns a contiguous band of
// tiles, and most halo rows and columns it reads sit in its own L2.
// Workgroups past the last tile are idle (no loads or stores, zero partials).
struct TileXY {
  int i0;     // first column of the tile
  int j0;     // first row of this wavefront
  bool valid;
};

// b: the workgroup's index within its solve; a solve's workgroups start at a
// multiple of 8 in the launch, so b % 8 is still the XCD.
__device__ __forceinline__ TileXY tile_xy_at(int nx, int ny, int R, int b) {
  const int gxt = (nx + kWave - 1) / kWave;
  const int gyt = (ny + kWaves * R - 1) / (kWaves * R);
  const int T = gxt * gyt;
  const int per = (T + 7) / 8;
  int t = (b & 7) * per + (b >> 3);
  TileXY o;
  o.valid = t < T;
  if (!o.valid) t = 0;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  o.i0 = (t % gxt) * kWave;
  o.j0 = ((t / gxt) * kWaves + w) * R;
  return o;
}

__device__ __forceinline__ TileXY tile_xy(int nx, int ny, int R) { return tile_xy_at(nx, ny, R, blockIdx.x); }

__device__ __forceinline__ int block_linear() { return blockIdx.x; }

// Register tile of one wavefront: rows j0-1 .. j0+R of its own column and
// rows j0 .. j0+R-1 of its halo column (lanes 0 and 63). All loads of a tile
// are issued together, before any dependent arithmetic.
template <typename T, int R>
struct Tile {
  T own[R + 2];
  T halo[R];
};

struct ColIdx {
  int i, ih;
  bool ok, hok;
};

__device__ __forceinline__ ColIdx col_idx(int nx, const TileXY& tl) {
  ColIdx c;
  const int lane = threadIdx.x & (kWave - 1);
  c.i = tl.i0 + lane;
  c.ok = tl.valid && c.i < nx;
  c.ih = (lane == 0) ? c.i - 1 : c.i + 1;
  c.hok = tl.valid && (lane == 0 || lane == kWave - 1) && c.ih >= 0 && c.ih < nx;
  return c;
}

// Tile loads are raw buffer loads: an offset at or beyond the buffer's size
// returns 0 in hardware, so rows and columns off the grid need no branches
// and every load of a tile issues back to back.
constexpr uint32_t kOOB = 0x80000000u;  // offset that is out of range for any buffer < 2 GiB

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

// A pointer loaded from device memory that is the same in every lane, moved
// to scalar registers. The compiler cannot always prove such a load uniform;
// a buffer descriptor built from a vector register would make every buffer
// access a loop over the distinct descriptors.
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return (T*)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}

__device__ __forceinline__ double bload64(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

__device__ __forceinline__ void bstore64(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
  using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, (int)off, 0, 0);
}

// Byte offset of an FP64 cell (kOOB off the grid); a problem holds at most
// 2^28 cells, so every in-grid offset of an FP64 array is below 2^31.
__device__ __forceinline__ uint32_t cell_off8(bool ok, int j, int ny, int nx, int i) {
  return (ok && j >= 0 && j < ny) ? (uint32_t)(j * nx + i) * 8u : kOOB;
}

// Buffer store: the hardware drops a store whose offset is out of range, so
// cells off the grid need no branch (pass kOOB).
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)off, 0, 0);
}

__device__ __forceinline__ uint32_t cell_off(bool ok, int j, int ny, int nx, int i) {
  return (ok && j >= 0 && j < ny) ? (uint32_t)(j * nx + i) * 4u : kOOB;
}

template <int R>
__device__ __forceinline__ void load_tile(__amdgpu_buffer_rsrc_t v, int nx, int ny, int j0, const ColIdx& c,
                                          Tile<float, R>& t) {
#pragma unroll
  for (int q = 0; q < R + 2; ++q) t.own[q] = bload(v, cell_off(c.ok, j0 - 1 + q, ny, nx, c.i));
#pragma unroll
  for (int q = 0; q < R; ++q) t.halo[q] = bload(v, cell_off(c.hok, j0 + q, ny, nx, c.ih));
}

template <int R>
__device__ __forceinline__ void load_rows_own(__amdgpu_buffer_rsrc_t v, int nx, int ny, int j0, const ColIdx& c,
                                              float (&out)[R]) {
#pragma unroll
  for (int q = 0; q < R; ++q) out[q] = bload(v, cell_off(c.ok, j0 + q, ny, nx, c.i));
}

// Wave-uniform row coefficients for rows j0-1 .. j0+R: hy (R+2 values) and the
// faces gy[j0-1 .. j0+R+1] (R+3 values); the padded arrays read 0 off the grid.
template <typename T, int R>
struct RowCoef {
  T hy[R + 2];
  T gy[R + 3];
};

template <typename T, int R>
__device__ __forceinline__ void load_rows(const T* __restrict__ hy, const T* __restrict__ gy, int j0,
                                          RowCoef<T, R>& rc) {
#pragma unroll
  for (int q = 0; q < R + 2; ++q) rc.hy[q] = hy[j0 - 1 + q];
#pragma unroll
  for (int q = 0; q < R + 3; ++q) rc.gy[q] = gy[j0 - 1 + q];
}

// Column coefficients of the own column and the halo column (padded arrays:
// columns -1 .. nx + 63 are readable and 0 off the grid).
template <typename T>
struct ColCoef {
  T hx, gw, ge, hxh, gwh, geh;
};

template <typename T>
__device__ __forceinline__ ColCoef<T> load_cols(const T* __restrict__ hx, const T* __restrict__ gx,
                                                const ColIdx& c) {
  ColCoef<T> k;
  k.hx = hx[c.i];
  k.gw = gx[c.i];
  k.ge = gx[c.i + 1];
  k.hxh = hx[c.ih];
  k.gwh = gx[c.ih];
  k.geh = gx[c.ih + 1];
  return k;
}

// y = A v on the R rows of the tile; own[q + 1] is the centre of output row q.
template <typename T, int R>
__device__ __forceinline__ void stencil_rows(const Tile<T, R>& v, const RowCoef<T, R>& rc, const ColCoef<T>& k,
                                             T (&out)[R]) {
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const T vc = v.own[q + 1];
    T ve, vw;
    east_west(vc, v.halo[q], ve, vw);
    out[q] = stencil5(vc, ve, vw, v.own[q + 2], v.own[q], rc.hy[q + 1], rc.gy[q + 1], rc.gy[q + 2], k.hx,
                      k.gw, k.ge);
  }
}

// The solid-mask operator on the R rows of the tile: face terms weighted by
// the neighbour's fluid flag, the sum by the own cell's, and x itself on solid
// cells. m holds the fluid flags (0 or 1) in the tile's layout.
template <int R>
__device__ __forceinline__ void stencil_rows_masked(const Tile<float, R>& v, const Tile<float, R>& m,
                                                    const RowCoef<float, R>& rc, const ColCoef<float>& k,
                                                    float (&out)[R]) {
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const float vc = v.own[q + 1], mc = m.own[q + 1];
    float ve, vw, me, mw;
    east_west(vc, v.halo[q], ve, vw);
    east_west(mc, m.halo[q], me, mw);
    const float s = rc.hy[q + 1] * (k.ge * me * (vc - ve) + k.gw * mw * (vc - vw)) +
                    k.hx * (rc.gy[q + 2] * m.own[q + 2] * (vc - v.own[q + 2]) +
                            rc.gy[q + 1] * m.own[q] * (vc - v.own[q]));
    out[q] = mc * s + (1.f - mc) * vc;
  }
}

// FP64 sum over a wavefront on DPP lane moves (no LDS traffic): within each
// row of 16 lanes, quad xor 1, quad xor 2, half-row mirror and row mirror
// leave the row sum in every lane of the row (each step adds commuted equal
// pairs, so all lanes hold the same bits); the four row sums are then added
// in a fixed order. Every lane returns the same value.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xf, 0xf, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return ((readlane_f64(v, 0) + readlane_f64(v, 16)) + readlane_f64(v, 32)) + readlane_f64(v, 48);
}

// Fixed-order reduction of N partial arrays ([N][P]); every workgroup obtains
// the same bits. lds holds N * kWaves doubles.
template <int N>
__device__ __forceinline__ void reduce_sums(const double* __restrict__ part, int P, double* lds, double (&out)[N]) {
  double v[N];
#pragma unroll
  for (int m = 0; m < N; ++m) v[m] = 0.0;
  for (int k = threadIdx.x; k < P; k += kBlock) {
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] += part[(size_t)m * P + k];
  }
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
  for (int m = 0; m < N; ++m) v[m] = wave_sum_dpp(v[m]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int m = 0; m < N; ++m) lds[m * kWaves + w] = v[m];
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < N; ++m)
    out[m] = ((lds[m * kWaves] + lds[m * kWaves + 1]) + lds[m * kWaves + 2]) + lds[m * kWaves + 3];
}

// Workgroup sums of N values, stored by thread 0 into part[.][blk] ([N][P]).
template <int N>
__device__ __forceinline__ void store_sums(double (&v)[N], double* lds, double* __restrict__ part, int P, int blk) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
  for (int m = 0; m < N; ++m) v[m] = wave_sum_dpp(v[m]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int m = 0; m < N; ++m) lds[m * kWaves + w] = v[m];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int m = 0; m < N; ++m)
      part[(size_t)m * P + blk] =
          ((lds[m * kWaves] + lds[m * kWaves + 1]) + lds[m * kWaves + 2]) + lds[m * kWaves + 3];
  }
}

// FP64 sum over each row of 16 lanes (quad xor 1, quad xor 2, half-row
// mirror, row mirror); every lane of the row gets the row's sum.
__device__ __forceinline__ double row_sum16(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x141>(v);
  v += dpp_f64<0x140>(v);
  return v;
}

// Fixed-order reduction of N partial arrays ([N][P]) in every workgroup, with
// one 16-lane row per sum: thread 16m + c adds the partials k = c, c + 16, ...
// of sum m (four running sums over k mod 64, then added in order), the row
// adds its 16 values, and thread 16m leaves the total in lds[m]; all threads
// then read the N totals. Every workgroup does the same operations in the
// same order, so all obtain the same bits. Needs 16 N <= kBlock.
template <int N>
__device__ __forceinline__ void reduce_sums16(const double* __restrict__ part, int P, double* lds, double (&out)[N]) {
  static_assert(16 * N <= kBlock, "one 16-lane row per sum");
  const int t = threadIdx.x;
  if (t < 16 * N) {
    const int m = t >> 4, c = t & 15;
    const double* __restrict__ pm = part + (size_t)m * P;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int k = c;
    for (; k + 48 < P; k += 64) {
      a0 += pm[k];
      a1 += pm[k + 16];
      a2 += pm[k + 32];
      a3 += pm[k + 48];
    }
    if (k < P) a0 += pm[k];
    if (k + 16 < P) a1 += pm[k + 16];
    if (k + 32 < P) a2 += pm[k + 32];
    const double v = row_sum16(((a0 + a1) + a2) + a3);
    if (c == 0) lds[m] = v;
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < N; ++m) out[m] = lds[m];
}

// The same reduction split in two, so that a kernel can issue the loads of
// the partials before its own tile loads: loads complete in issue order, and
// the scalars that the tile's arithmetic needs then arrive first.
// sums16_load: thread 16m + c loads partials k = c + 16 i (i < K) of sum m
// (0 past P; part is [N][P]). sums16_finish: adds them in order of i, then
// any partials past 16 K, and finishes as reduce_sums16. The order is fixed
// for a given P, so every workgroup obtains the same bits.
template <int N, int K>
__device__ __forceinline__ void sums16_load(const double* __restrict__ part, int P, double (&pre)[K]) {
  static_assert(16 * N <= kBlock, "one 16-lane row per sum");
  const int t = threadIdx.x;
  const int m = t >> 4, c = t & 15;
  const auto rs = make_rsrc(part, (uint64_t)N * P * 8);
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const int k = c + 16 * i;
    pre[i] = bload64(rs, (t < 16 * N && k < P) ? (uint32_t)(m * P + k) * 8u : kOOB);
  }
}

template <int N, int K>
__device__ __forceinline__ void sums16_finish(const double* __restrict__ part, int P, const double (&pre)[K],
                                              double* lds, double (&out)[N]) {
  const int t = threadIdx.x;
  if (t < 16 * N) {
    const int m = t >> 4, c = t & 15;
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < K; ++i) v += pre[i];
    for (int k = c + 16 * K; k < P; k += 16) v += part[(size_t)m * P + k];
    v = row_sum16(v);
    if (c == 0) lds[m] = v;
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < N; ++m) out[m] = lds[m];
}

template <typename T>
__device__ __forceinline__ T diag_of(T hyj, T gs, T gn, T hx, T gw, T ge) {
  return hyj * (gw + ge) + hx * (gs + gn);
}

// Jacobi preconditioner of this iteration form: z = r * dinv with dinv the
// hardware reciprocal of the diagonal (one rounding of 1/D, the same value in
// every launch, so the preconditioner is a fixed diagonal matrix). Cells off
// the grid have D = 0 and r = 0, and get z = 0.
__device__ __forceinline__ float inv_diag(float hyj, float gs, float gn, float hx, float gw, float ge) {
  return __builtin_amdgcn_rcpf(fmaxf(diag_of(hyj, gs, gn, hx, gw, ge), 1e-30f));
}

// FP64 true residual r = b - A x at (i, j) with b = hx hy f - mean(b); x
// holds the centre and its four neighbours.
__device__ __forceinline__ double true_res(const Coef& c, int i, int j, double xc_, double xe, double xw, double xn,
                                           double xs, float f, double bmean) {
  const double hyj = c.hy64[j];
  const double Ax = stencil5(xc_, xe, xw, xn, xs, hyj, c.gy64[j], c.gy64[j + 1], c.hx64[i], c.gx64[i],
                             c.gx64[i + 1]);
  return (c.hx64[i] * hyj * (double)f - bmean) - Ax;
}

}  // namespace ppe
