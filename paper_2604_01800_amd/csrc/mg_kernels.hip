// Multigrid V-cycle kernels (HIP, gfx950): the preconditioner of the MGPCG
// CG-type (Sec. 2.5, four levels by default).
//
// Level l+1 merges 2 x 2 cells of level l; prolongation is piecewise
// constant and restriction its transpose (sum over the four children), and
// the coarse operators are the Galerkin products P^T A P, which on a tensor
// grid are again five-point operators of 1D arrays (merged widths, the fine
// face factors at surviving faces), so every level runs the same matrix-free
// stencil. Smoothing is the degree-2 Chebyshev semi-iteration on D^-1 A over
// [0.2, 2] (Saad, Sec. 12.3), before the coarse correction from a zero guess
// and after it:
//   pre:   x1 = D^-1 b / theta;  r1 = b - A x1;
//          x2 = x1 + c1 x1 + c2 D^-1 r1
//   post:  x3 = x2 + P e;  r3 = b - A x3;  d = D^-1 r3 / theta;  x4 = x3 + d;
//          r4 = b - A x4;  x5 = x4 + c1 d + c2 D^-1 r4
// with theta, delta the interval's centre and half-width, c1 = rho1 rho0,
// c2 = 2 rho1 / delta (rho0 = delta / theta, rho1 = 1 / (2 theta/delta - rho0)).
// Each kernel recomputes what it needs on a one-cell halo, so a level costs
// four launches: pre-smoothing, residual + restriction, prolongation + first
// post step, second post step. A kernel that reads a vector on a halo never
// writes that vector (other workgroups may still be reading it): x2 and x5
// live in x, x4 in y. The coarsest level is solved exactly by the
// separable direct method (transforms to the eigenbases of both axes, a
// diagonal scaling, and back) in FP64, with the right-hand side's mean removed
// before and the solution's mean after, i.e. the minimum-norm solution.
//
// Vectors are FP32; every kernel returns at once for a solve whose done flag
// is set. The last kernel of the fine level leaves the partial sums of r.z in
// the PCG's partial-sum array, tiled as its phase kernels are.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"
#include "mg_internal.hpp"
#include "stencil.hpp"

namespace ppe {

namespace {

struct Cheb {
  float inv_theta, c1, c2;
};

Cheb cheb_consts() {
  const double theta = 0.5 * (kChebHi + kChebLo), delta = 0.5 * (kChebHi - kChebLo);
  const double sigma = theta / delta;
  const double rho0 = 1.0 / sigma, rho1 = 1.0 / (2.0 * sigma - rho0);
  return Cheb{(float)(1.0 / theta), (float)(rho1 * rho0), (float)(2.0 * rho1 / delta)};
}

// Arguments of one level's kernels (passed by value).
struct LevelArgs {
  Coef c;
  int64_t N;               // cells per solve on this level
  const float* b;          // [nb][N]
  float* x;                // [nb][N] x2, then x5
  float* y;                // [nb][N] x4
  float* d;                // [nb][N]
  const int32_t* flags;    // [nb] done codes of the solves
  Cheb k;
  // restriction target / coarse correction source (level l+1)
  float* bc;               // [nb][Nc] coarse right-hand side
  const float* ec;         // [nb][Nc] coarse solution
  int nxc;
  int64_t Nc;
  int coarsest;            // level l+1 is the coarsest: means are taken there
  double* bpart;           // [nb][P] partial sums of the coarse right-hand side (coarsest only)
  const double* xpart;     // [nb][nyc] row sums of the coarsest solution (coarsest only)
  int nyc;
  double* rzpart;          // fine level: partial sums of r.z, PCG layout (stride 2 P per solve), else NULL
  int P;                   // workgroups per solve of this level
};

}  // namespace

__device__ __forceinline__ float dinv_at(float hyj, float gs, float gn, float hx, float gw, float ge) {
  return 1.0f / fmaxf(diag_of(hyj, gs, gn, hx, gw, ge), 1e-30f);
}

// Pre-smoothing from a zero guess: writes x2.
template <int R>
__global__ __launch_bounds__(kBlock) void k_mg_pre(LevelArgs a) {
  const int s = blockIdx.z, nx = a.c.nx, ny = a.c.ny;
  if (a.flags[s] != DONE_NO) return;
  const size_t off = (size_t)s * a.N;
  const uint64_t vbytes = (uint64_t)a.N * 4;
  const TileXY tl = tile_xy(nx, ny, R);
  const ColIdx ci = col_idx(nx, tl);
  const int j0 = tl.j0;
  Tile<float, R> tb;
  load_tile<R>(make_rsrc(a.b + off, vbytes), nx, ny, j0, ci, tb);
  RowCoef<float, R> rc;
  load_rows<float, R>(a.c.hy, a.c.gy, j0, rc);
  const ColCoef<float> k = load_cols<float>(a.c.hx, a.c.gx, ci);
  Tile<float, R> x1;
  float dv[R];
#pragma unroll
  for (int q = 0; q < R + 2; ++q) {
    const float di = dinv_at(rc.hy[q], rc.gy[q], rc.gy[q + 1], k.hx, k.gw, k.ge);
    x1.own[q] = tb.own[q] * di * a.k.inv_theta;
    if (q >= 1 && q <= R) dv[q - 1] = di;
  }
#pragma unroll
  for (int q = 0; q < R; ++q)
    x1.halo[q] = tb.halo[q] * dinv_at(rc.hy[q + 1], rc.gy[q + 1], rc.gy[q + 2], k.hxh, k.gwh, k.geh) * a.k.inv_theta;
  float Ax[R];
  stencil_rows<float, R>(x1, rc, k, Ax);
  const auto xs = make_rsrc(a.x + off, vbytes);
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const float r1 = tb.own[q + 1] - Ax[q];
    const float x2 = x1.own[q + 1] + a.k.c1 * x1.own[q + 1] + a.k.c2 * dv[q] * r1;
    bstore(xs, cell_off(ci.ok, j0 + q, ny, nx, ci.i), x2);
  }
}

// Residual of x2 and its restriction (sum over 2 x 2 children) to the coarse
// right-hand side; on the way to the coarsest level also the partial sums of
// the coarse right-hand side (its mean is removed there).
template <int R>
__global__ __launch_bounds__(kBlock) void k_mg_restrict(LevelArgs a) {
  __shared__ double lds[kWaves];
  const int s = blockIdx.z, nx = a.c.nx, ny = a.c.ny;
  if (a.flags[s] != DONE_NO) return;
  const size_t off = (size_t)s * a.N;
  const uint64_t vbytes = (uint64_t)a.N * 4;
  const TileXY tl = tile_xy(nx, ny, R);
  const ColIdx ci = col_idx(nx, tl);
  const int j0 = tl.j0;
  Tile<float, R> tx;
  float bv[R];
  load_tile<R>(make_rsrc(a.x + off, vbytes), nx, ny, j0, ci, tx);
  load_rows_own<R>(make_rsrc(a.b + off, vbytes), nx, ny, j0, ci, bv);
  RowCoef<float, R> rc;
  load_rows<float, R>(a.c.hy, a.c.gy, j0, rc);
  const ColCoef<float> k = load_cols<float>(a.c.hx, a.c.gx, ci);
  float Ax[R];
  stencil_rows<float, R>(tx, rc, k, Ax);
  const int lane = threadIdx.x & (kWave - 1);
  const auto cs = make_rsrc(a.bc + (size_t)s * a.Nc, (uint64_t)a.Nc * 4);
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < R; q += 2) {
    // rows j0+q and j0+q+1 form one coarse row (j0 and R are even); off the
    // grid both the residual's inputs and its coefficients are 0
    const float v = (bv[q] - Ax[q]) + (bv[q + 1] - Ax[q + 1]);
    float ve, vw;
    east_west(v, 0.f, ve, vw);
    const float sum = v + ve;  // columns i and i+1 (i even; the pair never crosses a 64-column strip)
    const int j = j0 + q;
    const bool w = ci.ok && (lane & 1) == 0 && j < ny;
    bstore(cs, w ? (uint32_t)((j >> 1) * a.nxc + (ci.i >> 1)) * 4u : kOOB, sum);
    if (w) acc += (double)sum;
  }
  if (a.coarsest) {
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) a.bpart[(size_t)s * a.P + block_linear()] = acc;
  }
}

// Coarse correction and the first post-smoothing step: x3 = x2 + P e,
// d = D^-1 (b - A x3) / theta, x4 = x3 + d; reads x2 from x, writes x4 to y
// and d.
template <int R>
__global__ __launch_bounds__(kBlock) void k_mg_post1(LevelArgs a) {
  __shared__ double lds[kWaves];
  const int s = blockIdx.z, nx = a.c.nx, ny = a.c.ny;
  if (a.flags[s] != DONE_NO) return;
  const size_t off = (size_t)s * a.N;
  const uint64_t vbytes = (uint64_t)a.N * 4;
  const TileXY tl = tile_xy(nx, ny, R);
  const ColIdx ci = col_idx(nx, tl);
  const int j0 = tl.j0;
  Tile<float, R> tx;
  float bv[R];
  load_tile<R>(make_rsrc(a.x + off, vbytes), nx, ny, j0, ci, tx);
  load_rows_own<R>(make_rsrc(a.b + off, vbytes), nx, ny, j0, ci, bv);
  // coarse values of the parents of the tile's cells (0 off the grid)
  const auto es = make_rsrc(a.ec + (size_t)s * a.Nc, (uint64_t)a.Nc * 4);
  Tile<float, R> te;
#pragma unroll
  for (int q = 0; q < R + 2; ++q) {
    const int j = j0 - 1 + q;
    te.own[q] = bload(es, (ci.ok && j >= 0 && j < ny) ? (uint32_t)((j >> 1) * a.nxc + (ci.i >> 1)) * 4u : kOOB);
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int j = j0 + q;
    te.halo[q] = bload(es, (ci.hok && j < ny) ? (uint32_t)((j >> 1) * a.nxc + (ci.ih >> 1)) * 4u : kOOB);
  }
  RowCoef<float, R> rc;
  load_rows<float, R>(a.c.hy, a.c.gy, j0, rc);
  const ColCoef<float> k = load_cols<float>(a.c.hx, a.c.gx, ci);
  float emean = 0.f;
  if (a.coarsest) {
    // minimum-norm coarsest solution: subtract its plain mean (fixed-order sum)
    double sum = 0.0;
    for (int t = threadIdx.x; t < a.nyc; t += kBlock) sum += a.xpart[(size_t)s * a.nyc + t];
    emean = (float)(block_sum(sum, lds) / (double)a.Nc);
  }
  Tile<float, R> x3;
#pragma unroll
  for (int q = 0; q < R + 2; ++q) {
    const int j = j0 - 1 + q;
    const bool in = ci.ok && j >= 0 && j < ny;
    x3.own[q] = tx.own[q] + (in ? te.own[q] - emean : 0.f);
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const bool in = ci.hok && j0 + q < ny;
    x3.halo[q] = tx.halo[q] + (in ? te.halo[q] - emean : 0.f);
  }
  float Ax[R];
  stencil_rows<float, R>(x3, rc, k, Ax);
  const auto xs = make_rsrc(a.y + off, vbytes);
  const auto ds = make_rsrc(a.d + off, vbytes);
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const float di = dinv_at(rc.hy[q + 1], rc.gy[q + 1], rc.gy[q + 2], k.hx, k.gw, k.ge);
    const float dd = (bv[q] - Ax[q]) * di * a.k.inv_theta;
    const uint32_t o = cell_off(ci.ok, j0 + q, ny, nx, ci.i);
    bstore(xs, o, x3.own[q + 1] + dd);
    bstore(ds, o, dd);
  }
}

// Second post-smoothing step: x5 = x4 + c1 d + c2 D^-1 (b - A x4); reads x4
// from y, writes x5 to x. On the fine level b is the PCG residual r and x5
// is z; the workgroup's share of r.z goes to the PCG's partial sums.
template <int R>
__global__ __launch_bounds__(kBlock) void k_mg_post2(LevelArgs a) {
  __shared__ double lds[kWaves];
  const int s = blockIdx.z, nx = a.c.nx, ny = a.c.ny;
  if (a.flags[s] != DONE_NO) return;
  const size_t off = (size_t)s * a.N;
  const uint64_t vbytes = (uint64_t)a.N * 4;
  const TileXY tl = tile_xy(nx, ny, R);
  const ColIdx ci = col_idx(nx, tl);
  const int j0 = tl.j0;
  Tile<float, R> tx;
  float bv[R], dv[R];
  load_tile<R>(make_rsrc(a.y + off, vbytes), nx, ny, j0, ci, tx);
  load_rows_own<R>(make_rsrc(a.b + off, vbytes), nx, ny, j0, ci, bv);
  load_rows_own<R>(make_rsrc(a.d + off, vbytes), nx, ny, j0, ci, dv);
  RowCoef<float, R> rc;
  load_rows<float, R>(a.c.hy, a.c.gy, j0, rc);
  const ColCoef<float> k = load_cols<float>(a.c.hx, a.c.gx, ci);
  float Ax[R];
  stencil_rows<float, R>(tx, rc, k, Ax);
  const auto xs = make_rsrc(a.x + off, vbytes);
  double rz = 0.0;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const float di = dinv_at(rc.hy[q + 1], rc.gy[q + 1], rc.gy[q + 2], k.hx, k.gw, k.ge);
    const float x5 = tx.own[q + 1] + a.k.c1 * dv[q] + a.k.c2 * di * (bv[q] - Ax[q]);
    const uint32_t o = cell_off(ci.ok, j0 + q, ny, nx, ci.i);
    bstore(xs, o, x5);
    if (o != kOOB) rz += (double)bv[q] * (double)x5;
  }
  if (a.rzpart) {
    rz = block_sum(rz, lds);
    if (threadIdx.x == 0) a.rzpart[(size_t)s * 2 * a.P + block_linear()] = rz;
  }
}

// r.z partial sums when the fine level is itself the coarsest (one level).
template <int R>
__global__ __launch_bounds__(kBlock) void k_mg_rz(LevelArgs a) {
  __shared__ double lds[kWaves];
  const int s = blockIdx.z, nx = a.c.nx, ny = a.c.ny;
  if (a.flags[s] != DONE_NO) return;
  const size_t off = (size_t)s * a.N;
  const uint64_t vbytes = (uint64_t)a.N * 4;
  const TileXY tl = tile_xy(nx, ny, R);
  const ColIdx ci = col_idx(nx, tl);
  const int j0 = tl.j0;
  float bv[R], xv[R];
  load_rows_own<R>(make_rsrc(a.b + off, vbytes), nx, ny, j0, ci, bv);
  load_rows_own<R>(make_rsrc(a.x + off, vbytes), nx, ny, j0, ci, xv);
  double rz = 0.0;
#pragma unroll
  for (int q = 0; q < R; ++q) rz += (double)bv[q] * (double)xv[q];
  rz = block_sum(rz, lds);
  if (threadIdx.x == 0) a.rzpart[(size_t)s * 2 * a.P + block_linear()] = rz;
}

namespace {
struct CoarseArgs {
  int nxc, nyc;
  int64_t Nc;
  const float* b;        // [nb][Nc]
  float* x;              // [nb][Nc]
  const double* phi;     // [nxc][nxc]
  const double* phiT;    // [nxc][nxc]
  const double* psi;     // [nyc][nyc]
  const double* psiT;    // [nyc][nyc]
  const double* dinv;    // [nyc][nxc]
  double* bh;            // [nb][nyc][nxc]
  const double* bpart;   // [nb][bP] or NULL
  int bP;
  double* xpart;         // [nb][nyc]
  const int32_t* flags;
};
}  // namespace

// sum_q M[q * ld + j] v[q] for q < n (v in LDS), accumulated in q order.
// The matrix loads of 32 terms are issued together before their products, so
// the sum waits for the L2 once per 32 terms instead of once per few.
__device__ __forceinline__ double dot_strided(const double* __restrict__ M, int ld, int j, const double* v, int n) {
  constexpr int B = 32;
  double acc = 0.0;
  int q0 = 0;
  for (; q0 + B <= n; q0 += B) {
    double m[B];
#pragma unroll
    for (int u = 0; u < B; ++u) m[u] = M[(size_t)(q0 + u) * ld + j];
#pragma unroll
    for (int u = 0; u < B; ++u) acc += m[u] * v[q0 + u];
  }
  for (; q0 < n; ++q0) acc += M[(size_t)q0 * ld + j] * v[q0];
  return acc;
}

// Row transform of the coarsest right-hand side (its mean removed):
// bh[j][k] = sum_i phi[i][k] b[j][i]; one workgroup per row.
__global__ __launch_bounds__(kBlock) void k_mg_cfwd(CoarseArgs a) {
  extern __shared__ double row[];
  __shared__ double lds[kWaves];
  const int s = blockIdx.z, j = blockIdx.x;
  if (a.flags[s] != DONE_NO) return;
  double mean = 0.0;
  if (a.bpart) mean = reduce_partials(a.bpart + (size_t)s * a.bP, a.bP, lds) / (double)a.Nc;
  const float* b = a.b + (size_t)s * a.Nc + (size_t)j * a.nxc;
  for (int i = threadIdx.x; i < a.nxc; i += kBlock) row[i] = (double)b[i] - mean;
  __syncthreads();
  double* out = a.bh + (size_t)s * a.Nc + (size_t)j * a.nxc;
  for (int k = threadIdx.x; k < a.nxc; k += kBlock) out[k] = dot_strided(a.phi, a.nxc, k, row, a.nxc);
}

// Column k of the transformed right-hand side: forward transform along y
// (bh[j][k] <- sum_j' psi[j'][j] bh[j'][k]), division by lam_k + mu_j, and the
// inverse transform along y (bh[j][k] <- sum_j' psi[j][j'] c[j'][k]); one
// workgroup per column, in place (no other workgroup touches the column).
__global__ __launch_bounds__(kBlock) void k_mg_ccol(CoarseArgs a) {
  extern __shared__ double col[];  // [2][nyc]
  const int s = blockIdx.z, k = blockIdx.x;
  if (a.flags[s] != DONE_NO) return;
  const int n = a.nyc, m = a.nxc;
  double* c = a.bh + (size_t)s * a.Nc + k;
  double* t = col;
  double* u = col + n;
  for (int j = threadIdx.x; j < n; j += kBlock) t[j] = c[(size_t)j * m];
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += kBlock) u[j] = dot_strided(a.psi, n, j, t, n) * a.dinv[(size_t)j * m + k];
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += kBlock) c[(size_t)j * m] = dot_strided(a.psiT, n, j, u, n);
}

// Back-transform x[j][i] = sum_k phi[i][k] c[j][k] and the row sums of x (the
// fine level's prolongation removes the mean); one workgroup per row.
__global__ __launch_bounds__(kBlock) void k_mg_cbwd(CoarseArgs a) {
  extern __shared__ double row[];
  __shared__ double lds[kWaves];
  const int s = blockIdx.z, j = blockIdx.x;
  if (a.flags[s] != DONE_NO) return;
  const double* c = a.bh + (size_t)s * a.Nc + (size_t)j * a.nxc;
  for (int k = threadIdx.x; k < a.nxc; k += kBlock) row[k] = c[k];
  __syncthreads();
  float* x = a.x + (size_t)s * a.Nc + (size_t)j * a.nxc;
  double sum = 0.0;
  for (int i = threadIdx.x; i < a.nxc; i += kBlock) {
    const double acc = dot_strided(a.phiT, a.nxc, i, row, a.nxc);
    x[i] = (float)acc;
    sum += (double)(float)acc;
  }
  sum = block_sum(sum, lds);
  if (threadIdx.x == 0) a.xpart[(size_t)s * a.nyc + j] = sum;
}

// ---------------------------------------------------------------------------
#define PPE_MG_DISPATCH(R, ...)                                  \
  switch (R) {                                                   \
    case 2: { constexpr int RR = 2; __VA_ARGS__; } break;        \
    case 4: { constexpr int RR = 4; __VA_ARGS__; } break;        \
    case 8: { constexpr int RR = 8; __VA_ARGS__; } break;        \
    default: { constexpr int RR = 16; __VA_ARGS__; } break;      \
  }

void launch_vcycle(const PcgArgs& pa, int nb, hipStream_t s) {
  const MgData& m = *pa.mg;
  const int L = m.L;
  const Cheb k = cheb_consts();
  // level l's arguments; the fine level reads the PCG residual and writes z
  // with the PCG's tiling, so its r.z partials line up with phase A's sums
  auto level = [&](int l) {
    const MgLevel& v = m.lv[l];
    LevelArgs a{};
    a.c = v.c;
    a.N = (int64_t)v.nx * v.ny;
    a.b = l == 0 ? pa.r : v.b;
    a.x = l == 0 ? m.z : v.x;
    a.y = l == 0 ? m.y0 : v.y;
    a.d = l == 0 ? m.d0 : v.d;
    a.flags = pa.flags;
    a.k = k;
    if (l + 1 < L) {
      const MgLevel& c = m.lv[l + 1];
      a.bc = c.b;
      a.ec = c.x;
      a.nxc = c.nx;
      a.Nc = (int64_t)c.nx * c.ny;
      a.coarsest = l + 1 == L - 1;
      a.bpart = m.bpart;
      a.xpart = m.xpart;
      a.nyc = c.ny;
    }
    a.P = l == 0 ? pa.P : v.P;
    a.rzpart = l == 0 ? pa.partB + pa.P : nullptr;
    return a;
  };
  auto rows = [&](int l) { return l == 0 ? pa.R : m.lv[l].R; };
  for (int l = 0; l + 1 < L; ++l) {
    const LevelArgs a = level(l);
    const dim3 g = stencil_grid(a.c, rows(l), nb);
    PPE_MG_DISPATCH(rows(l), k_mg_pre<RR><<<g, kBlock, 0, s>>>(a); k_mg_restrict<RR><<<g, kBlock, 0, s>>>(a));
  }
  {
    const MgLevel& c = m.lv[L - 1];
    CoarseArgs ca{};
    ca.nxc = m.nxc;
    ca.nyc = m.nyc;
    ca.Nc = (int64_t)m.nxc * m.nyc;
    ca.b = L == 1 ? pa.r : c.b;
    ca.x = L == 1 ? m.z : c.x;
    ca.phi = m.phi;
    ca.phiT = m.phiT;
    ca.psi = m.psi;
    ca.psiT = m.psiT;
    ca.dinv = m.dinv;
    ca.bh = m.bh;
    ca.bpart = L == 1 ? nullptr : m.bpart;
    ca.bP = m.bP;
    ca.xpart = m.xpart;
    ca.flags = pa.flags;
    const size_t shm = sizeof(double) * m.nxc;
    k_mg_cfwd<<<dim3(m.nyc, 1, nb), kBlock, shm, s>>>(ca);
    k_mg_ccol<<<dim3(m.nxc, 1, nb), kBlock, sizeof(double) * 2 * m.nyc, s>>>(ca);
    k_mg_cbwd<<<dim3(m.nyc, 1, nb), kBlock, shm, s>>>(ca);
  }
  if (L == 1) {
    const LevelArgs a = level(0);
    const dim3 g = stencil_grid(a.c, pa.R, nb);
    PPE_MG_DISPATCH(pa.R, k_mg_rz<RR><<<g, kBlock, 0, s>>>(a));
    return;
  }
  for (int l = L - 2; l >= 0; --l) {
    const LevelArgs a = level(l);
    const dim3 g = stencil_grid(a.c, rows(l), nb);
    PPE_MG_DISPATCH(rows(l), k_mg_post1<RR><<<g, kBlock, 0, s>>>(a); k_mg_post2<RR><<<g, kBlock, 0, s>>>(a));
  }
}

}  // namespace ppe
