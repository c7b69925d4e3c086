// Incomplete-Cholesky preconditioner IC(0) in red-black ordering (the ICPCG
// CG-type of Sec. 2.5), applied with the two-phase PCG kernels' tiling.
//
// Cell (i, j) is red when i + j is even. Red cells couple only to black
// cells in the 5-point operator, so IC(0) of the operator with every red
// cell ordered before every black one has a closed form: L = [D_r^1/2, 0;
// A_br D_r^-1/2, S^1/2] with S = D_b - diag(A_br D_r^-1 A_rb), i.e.
// S_b = D_b - sum over the red neighbours r of w_br^2 / D_r (w the face
// weights). Both triangular solves of z = (L L^T)^-1 r then become passes
// over independent cells:
//   black pass:  z_b = (r_b + sum_r w_br r_r / D_r) / S_b
//   red pass:    z_r = (r_r + sum_b w_rb z_b) / D_r
// q holds 1/D on red cells and 1/S on black cells, built once per problem.
// The red pass also leaves the workgroup's share of r.z where phase A of the
// PCG reads it (the multigrid preconditioner's fine level does the same).
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"
#include "stencil.hpp"

namespace ppe {

namespace {

__device__ __forceinline__ bool is_red(int i, int j) { return ((i + j) & 1) == 0; }

// sum over the four faces of the face weight times the neighbour's value,
// on output row q of the tile
template <int R>
__device__ __forceinline__ float nb_sum(const Tile<float, R>& v, const RowCoef<float, R>& rc,
                                        const ColCoef<float>& k, int q) {
  float ve, vw;
  east_west(v.own[q + 1], v.halo[q], ve, vw);
  return rc.hy[q + 1] * (k.ge * ve + k.gw * vw) + k.hx * (rc.gy[q + 2] * v.own[q + 2] + rc.gy[q + 1] * v.own[q]);
}

}  // namespace

template <int R>
__global__ __launch_bounds__(kBlock) void k_ic_black(PcgArgs a) {
  const int s = blockIdx.z, nx = a.c.nx, ny = a.c.ny;
  if (a.flags[s] != DONE_NO) return;
  const size_t off = (size_t)s * a.N;
  const uint64_t vbytes = (uint64_t)a.N * 4;
  const TileXY tl = tile_xy(nx, ny, R);
  const ColIdx ci = col_idx(nx, tl);
  const int j0 = tl.j0;
  Tile<float, R> tr, tq;
  load_tile<R>(make_rsrc(a.r + off, vbytes), nx, ny, j0, ci, tr);
  load_tile<R>(make_rsrc(a.icq, vbytes), nx, ny, j0, ci, tq);
  RowCoef<float, R> rc;
  load_rows<float, R>(a.c.hy, a.c.gy, j0, rc);
  const ColCoef<float> k = load_cols<float>(a.c.hx, a.c.gx, ci);
  // r / D on red cells, 0 on black cells (off the grid the loads gave 0)
  Tile<float, R> tt;
#pragma unroll
  for (int q = 0; q < R + 2; ++q) tt.own[q] = is_red(ci.i, j0 - 1 + q) ? tr.own[q] * tq.own[q] : 0.f;
#pragma unroll
  for (int q = 0; q < R; ++q) tt.halo[q] = is_red(ci.ih, j0 + q) ? tr.halo[q] * tq.halo[q] : 0.f;
  const auto zs = make_rsrc(a.z + off, vbytes);
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int j = j0 + q;
    const float zb = (tr.own[q + 1] + nb_sum<R>(tt, rc, k, q)) * tq.own[q + 1];
    bstore(zs, is_red(ci.i, j) ? kOOB : cell_off(ci.ok, j, ny, nx, ci.i), zb);
  }
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_ic_red(PcgArgs a) {
  __shared__ double lds[kWaves];
  const int s = blockIdx.z, nx = a.c.nx, ny = a.c.ny;
  if (a.flags[s] != DONE_NO) return;
  const size_t off = (size_t)s * a.N;
  const uint64_t vbytes = (uint64_t)a.N * 4;
  const TileXY tl = tile_xy(nx, ny, R);
  const ColIdx ci = col_idx(nx, tl);
  const int j0 = tl.j0;
  Tile<float, R> tz;
  float rv[R], qv[R];
  load_tile<R>(make_rsrc(a.z + off, vbytes), nx, ny, j0, ci, tz);
  load_rows_own<R>(make_rsrc(a.r + off, vbytes), nx, ny, j0, ci, rv);
  load_rows_own<R>(make_rsrc(a.icq, vbytes), nx, ny, j0, ci, qv);
  RowCoef<float, R> rc;
  load_rows<float, R>(a.c.hy, a.c.gy, j0, rc);
  const ColCoef<float> k = load_cols<float>(a.c.hx, a.c.gx, ci);
  // the black pass's values; red entries of z are stale here
  Tile<float, R> tb;
#pragma unroll
  for (int q = 0; q < R + 2; ++q) tb.own[q] = is_red(ci.i, j0 - 1 + q) ? 0.f : tz.own[q];
#pragma unroll
  for (int q = 0; q < R; ++q) tb.halo[q] = is_red(ci.ih, j0 + q) ? 0.f : tz.halo[q];
  const auto zs = make_rsrc(a.z + off, vbytes);
  double rz = 0.0;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int j = j0 + q;
    const bool red = is_red(ci.i, j);
    const float zr = (rv[q] + nb_sum<R>(tb, rc, k, q)) * qv[q];
    const uint32_t o = cell_off(ci.ok, j, ny, nx, ci.i);
    bstore(zs, red ? o : kOOB, zr);
    if (o != kOOB) rz += (double)rv[q] * (double)(red ? zr : tb.own[q + 1]);
  }
  rz = block_sum(rz, lds);
  if (threadIdx.x == 0) a.partB[(size_t)s * 2 * a.P + a.P + block_linear()] = rz;
}

void launch_ic(const PcgArgs& a, int nb, hipStream_t s) {
  const dim3 g = stencil_grid(a.c, a.R, nb);
  switch (a.R) {
    case 2: k_ic_black<2><<<g, kBlock, 0, s>>>(a); k_ic_red<2><<<g, kBlock, 0, s>>>(a); break;
    case 4: k_ic_black<4><<<g, kBlock, 0, s>>>(a); k_ic_red<4><<<g, kBlock, 0, s>>>(a); break;
    case 8: k_ic_black<8><<<g, kBlock, 0, s>>>(a); k_ic_red<8><<<g, kBlock, 0, s>>>(a); break;
    default: k_ic_black<16><<<g, kBlock, 0, s>>>(a); k_ic_red<16><<<g, kBlock, 0, s>>>(a); break;
  }
}

}  // namespace ppe
