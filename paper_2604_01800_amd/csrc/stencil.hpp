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


}  // namespace ppe
