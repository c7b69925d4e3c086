// Single-reduction Jacobi-PCG: one launch and one grid-wide reduction per CG
// iteration (HIP, gfx950).
//
// The textbook PCG recurrences (Saad, Alg. 9.1; D = diag(A)) are regrouped so
// that a launch needs only the scalars reduced at the end of the launch
// before it. Given r_k, p_{k-1} and the sums over the grid
//   gamma_k = r_k.z_k,  delta_k = z_k.A z_k,  zeta_k = z_k.A p_{k-1},
//   pi_k = p_{k-1}.A p_{k-1}        (z = D^-1 r),
// one launch computes
//   beta_{k-1} = gamma_k / gamma_{k-1}                    (0 after a restart)
//   p_k        = z_k + beta_{k-1} p_{k-1}
//   p_k.A p_k  = delta_k + 2 beta zeta_k + beta^2 pi_k    (exact expansion)
//   alpha_k    = gamma_k / p_k.A p_k
//   x_c += alpha_k p_k,  s = A p_k,  r_{k+1} = r_k - alpha_k s
// and the partial sums of gamma, delta, zeta, pi and |r|^2 for k + 1. The
// expansion of p.Ap is an identity of bilinear forms, not a consequence of
// orthogonality, so the iterates equal the two-reduction form's in exact
// arithmetic. Each workgroup recomputes p on a two-cell halo and s, r_{k+1},
// z_{k+1} on a one-cell halo of its tile, which removes the second grid-wide
// dependency of the iteration. HBM traffic per cell: read r, p, x_c and
// write them (24 B); r and p alternate between two buffers by launch parity
// because neighbouring workgroups read their halos.
//
// Reliable updates take three launches: FLUSH adds x_c into the FP64
// solution, TRUE recomputes r = b - A x in FP64 on each tile with |r|^2 (the
// convergence judge), and SUMS forms the four sums of the next CG step from
// the stored true residual and the kept direction p. Each of them needs no
// more registers than the CG step, which keeps its occupancy. Every launch reads the state slots of the other parity, so no
// workgroup reads what the same launch writes.
#include <hip/hip_ext.h>

#include "common.hpp"
#include "kernels.hpp"
#include "stencil.hpp"

namespace ppe {

constexpr int kSums = 5;  // gamma, delta, zeta, pi, |r|^2

// Sums of solve s (of nbs solves sharing a.part1) written by launch parity par.
__device__ __forceinline__ double* sums_of(const PcgArgs& a, int par, int s, int nbs) {
  return a.part1 + ((size_t)par * nbs + s) * kSums * a.P;
}

// Halo columns in transposed form: lanes 0-31 work on the west side and
// lanes 32-63 on the east side of the wavefront's 64-column strip, one row
// per lane (lane t of a side takes row j0 - 1 + t). On each side, column e is
// the strip's edge column (i0 or i0 + 63), column h1 the first halo column
// (i0 - 1 or i0 + 64) and column h2 the second (i0 - 2 or i0 + 65). A lane
// loads and recomputes these few values itself, so the halo costs a handful
// of wavefront instructions instead of a full pass per halo row; the edge
// lanes 0 and 63 read the halo values back with readlane.
struct HaloT {
  int ce, c1, c2, j;         // columns and row of this lane's halo cell
  bool oke, ok1, ok2;        // columns on the grid (and the tile valid)
  bool east;                 // side
};

__device__ __forceinline__ HaloT halo_t(int nx, const TileXY& tl) {
  const int lane = threadIdx.x & (kWave - 1);
  HaloT h;
  h.east = lane >= 32;
  const int t = lane & 31;
  h.j = tl.j0 - 1 + t;
  h.ce = h.east ? tl.i0 + kWave - 1 : tl.i0;
  h.c1 = h.east ? tl.i0 + kWave : tl.i0 - 1;
  h.c2 = h.east ? tl.i0 + kWave + 1 : tl.i0 - 2;
  h.oke = tl.valid && h.ce < nx;
  h.ok1 = tl.valid && h.c1 >= 0 && h.c1 < nx;
  h.ok2 = tl.valid && h.c2 >= 0 && h.c2 < nx;
  return h;
}

// Value of the halo lane for side row q (west: lane q, east: lane 32 + q) in
// the edge lane of that side (lane 0 west, lane 63 east).
__device__ __forceinline__ float from_halo(float v, int q) {
  const int lane = threadIdx.x & (kWave - 1);
  const float w = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), q));
  const float e = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32 + q));
  return lane < 32 ? w : e;
}

// One launch of the iteration for solve s of the nbs solves described by a,
// run by the solve's workgroup blk.
template <int R, bool JAC>
__device__ __forceinline__ void pcg1_body(const PcgArgs& a, int s, int nbs, int blk, int par, double* lds) {
  const int nx = a.c.nx, ny = a.c.ny;
  SolveState* st = a.st + s;
  const int P = a.P, pm = par ^ 1;
  const size_t off = (size_t)s * a.N;
  const float* __restrict__ rin = (pm ? a.r1 : a.r) + off;
  float* __restrict__ rout = (par ? a.r1 : a.r) + off;
  const float* __restrict__ pin = (pm ? a.p1 : a.p0) + off;
  float* __restrict__ pout = (par ? a.p1 : a.p0) + off;
  float* __restrict__ xc = a.xc + off;
  const int lane = threadIdx.x & (kWave - 1);
  const TileXY tl = tile_xy_at(nx, ny, R, blk);
  const ColIdx ci = col_idx(nx, tl);
  const HaloT ht = halo_t(nx, tl);
  const int j0 = tl.j0;

  // Tile loads of the CG step first (they do not depend on the scalars): own
  // column rows j0-2 .. j0+R+1, and the transposed halo cells.
  const uint64_t vbytes = (uint64_t)a.N * 4;
  const auto rsr = make_rsrc(rin, vbytes), psr = make_rsrc(pin, vbytes);
  float ro[R + 4], po[R + 4], xcv[R];
#pragma unroll
  for (int q = 0; q < R + 4; ++q) {
    const uint32_t o = cell_off(ci.ok, j0 - 2 + q, ny, nx, ci.i);
    ro[q] = bload(rsr, o);
    po[q] = bload(psr, o);
  }
  const uint32_t oe = cell_off(ht.oke, ht.j, ny, nx, ht.ce), o1 = cell_off(ht.ok1, ht.j, ny, nx, ht.c1),
                 o2 = cell_off(ht.ok2, ht.j, ny, nx, ht.c2);
  const float hre = bload(rsr, oe), hpe = bload(psr, oe);
  const float hr1 = bload(rsr, o1), hp1 = bload(psr, o1);
  const float hr2 = bload(rsr, o2), hp2 = bload(psr, o2);
  load_rows_own<R>(make_rsrc(xc, vbytes), nx, ny, j0, ci, xcv);
  // Row coefficients of rows j0-2 .. j0+R+1 (faces j0-2 .. j0+R+2); padded arrays.
  float hy[R + 4], gy[R + 5];
#pragma unroll
  for (int q = 0; q < R + 4; ++q) hy[q] = a.c.hy[j0 - 2 + q];
#pragma unroll
  for (int q = 0; q < R + 5; ++q) gy[q] = a.c.gy[j0 - 2 + q];
  const ColCoef<float> k = load_cols<float>(a.c.hx, a.c.gx, ci);
  // the halo lane's row and columns
  const float hy_t = a.c.hy[ht.j], gs_t = a.c.gy[ht.j], gn_t = a.c.gy[ht.j + 1];
  const float hxe = a.c.hx[ht.ce], gwe = a.c.gx[ht.ce], gee = a.c.gx[ht.ce + 1];
  const float hx1 = a.c.hx[ht.c1], gw1 = a.c.gx[ht.c1], ge1 = a.c.gx[ht.c1 + 1];
  const float hx2 = a.c.hx[ht.c2], gw2 = a.c.gx[ht.c2], ge2 = a.c.gx[ht.c2 + 1];

  // State of the previous launch (never written by this launch).
  const int dprev = st->dflag[pm];
  const int pmode = st->mode[pm];
  const int max_iter = a.call->max_iter;
  const double delta2 = a.call->delta2;
  const int it = st->it[pm], nru = st->n_ru[pm], itcg = st->it_cg[pm];
  const int restart = st->restart[pm];
  const double gam_prev = st->rho[pm], thr2 = st->thr2;
  double rr_ru = st->rr_ru[pm];
  const bool leader = blk == 0 && threadIdx.x == 0;
  // Reduced whatever the previous mode (after a FLUSH the sums are stale and
  // unused), so that these loads do not wait for the mode word.
  double sum[kSums];
  reduce_sums<kSums>(sums_of(a, pm, s, nbs), P, lds, sum);
  if (__builtin_expect(dprev != 0, 0)) {
    if (leader) st->dflag[par] = dprev;
    return;
  }

  // What this launch does.
  int todo = MODE_CG, rst_next = 0;
  double alpha = 0.0, beta = 0.0;
  if (__builtin_expect(pmode == MODE_FLUSH, 0)) {
    todo = MODE_TRUE;
  } else if (__builtin_expect(pmode == MODE_TRUE, 0)) {
    // The last launch computed the FP64 true residual: judge convergence.
    const double rr = sum[4];
    int done = DONE_NO;
    if (!isfinite(rr)) done = DONE_NONFINITE;
    else if (rr <= thr2) done = DONE_CONV;
    else if (it >= max_iter) done = DONE_MAXIT;
    if (done) {
      if (leader) {
        st->rr_final = rr;
        st->it_final = it;
        st->nru_final = nru;
        st->itcg_final = itcg;
        st->done = done;
        st->t_done = wall_clock64();
        st->dflag[par] = done;
        a.flags[s] = done;
      }
      return;
    }
    todo = MODE_SUMS;
    rr_ru = rr;
  } else {
    // CG step from the sums of a CG or SUMS launch; after SUMS the residual is
    // fresh, so only a breakdown can send it back to a reliable update.
    const double gam = sum[0], del = sum[1], zet = sum[2], pip = sum[3], rr = sum[4];
    bool flush = pmode == MODE_CG && (!isfinite(rr) || rr <= thr2 || rr <= delta2 * rr_ru || it >= max_iter);
    if (!flush) {
      beta = (pmode == MODE_SUMS && restart) ? 0.0 : gam / gam_prev;
      if (!isfinite(beta)) beta = 0.0;
      const double pap = del + 2.0 * beta * zet + beta * beta * pip;
      alpha = gam / pap;
      if (!(pap > 0.0) || !isfinite(alpha)) {
        flush = true;  // breakdown: recompute the residual and restart
        rst_next = 1;
      }
    }
    if (flush) todo = MODE_FLUSH;
    if (leader && todo == MODE_CG) {
      st->mode[par] = MODE_CG;
      st->it[par] = it + 1;
      st->it_cg[par] = itcg + 1;
      st->n_ru[par] = nru;
      st->rho[par] = gam;
      st->rr_ru[par] = rr_ru;
      st->rr_last[par] = rr;
      st->restart[par] = 0;
      st->alpha[par] = alpha;
      st->dflag[par] = DONE_NO;
    }
  }

  if (__builtin_expect(todo == MODE_FLUSH, 0)) {
    // Reliable update, part 1: x += x_c in FP64, x_c = 0, p carried over.
    const auto xsr = make_rsrc(uniform_ptr(a.call->x) + off, (uint64_t)a.N * 8);
    const auto xcs = make_rsrc(xc, vbytes), pso = make_rsrc(pout, vbytes);
    double xv[R];
#pragma unroll
    for (int q = 0; q < R; ++q) xv[q] = bload64(xsr, cell_off8(ci.ok, j0 + q, ny, nx, ci.i));
#pragma unroll
    for (int q = 0; q < R; ++q) {
      bstore64(xsr, cell_off8(ci.ok, j0 + q, ny, nx, ci.i), xv[q] + (double)xcv[q]);
      const uint32_t o = cell_off(ci.ok, j0 + q, ny, nx, ci.i);
      bstore(xcs, o, 0.f);
      bstore(pso, o, po[q + 2]);
    }
    if (leader) {
      st->mode[par] = MODE_FLUSH;
      st->it[par] = it;
      st->it_cg[par] = itcg;
      st->n_ru[par] = nru + 1;
      st->rho[par] = gam_prev;
      st->rr_ru[par] = rr_ru;
      st->restart[par] = rst_next;
      st->dflag[par] = DONE_NO;
    }
    return;
  }

  double acc[kSums] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (__builtin_expect(todo == MODE_TRUE, 0)) {
    // Reliable update, part 2: r = b - A x in FP64 on the own rows (the x
    // window walks down the column; the halo column gives east/west), and
    // |r|^2 in FP64, the convergence judge. p is carried over.
    const auto xsr = make_rsrc(uniform_ptr(a.call->x) + off, (uint64_t)a.N * 8);
    const auto fsr = make_rsrc(uniform_ptr(a.call->f) + off, vbytes);
    const auto rso = make_rsrc(rout, vbytes), pso = make_rsrc(pout, vbytes);
    const double bmean = st->bmean;
    const auto psr2 = make_rsrc(pin, vbytes);
    double x_p = bload64(xsr, cell_off8(ci.ok, j0 - 1, ny, nx, ci.i));
    double x_c = bload64(xsr, cell_off8(ci.ok, j0, ny, nx, ci.i));
#pragma unroll 1
    for (int q = 0; q < R; ++q) {
      const int j = j0 + q;
      const double x_n = bload64(xsr, cell_off8(ci.ok, j + 1, ny, nx, ci.i));
      const double xh = bload64(xsr, cell_off8(ci.hok, j, ny, nx, ci.ih));
      const float fv = bload(fsr, cell_off(ci.ok, j, ny, nx, ci.i));
      double xe, xw;
      east_west(x_c, xh, xe, xw);
      const bool own_ok = ci.ok && j < ny;
      const double rv = true_res(a.c, ci.i, j, x_c, xe, xw, x_n, x_p, fv, bmean);
      const uint32_t o = cell_off(ci.ok, j, ny, nx, ci.i);
      bstore(rso, o, (float)rv);
      bstore(pso, o, bload(psr2, o));
      acc[4] += own_ok ? rv * rv : 0.0;
      x_p = x_c;
      x_c = x_n;
    }
    if (leader) {
      st->mode[par] = MODE_TRUE;
      st->it[par] = it;
      st->it_cg[par] = itcg;
      st->n_ru[par] = nru;
      st->rho[par] = gam_prev;
      st->rr_ru[par] = rr_ru;
      st->restart[par] = restart;
      st->dflag[par] = DONE_NO;
    }
  } else if (__builtin_expect(todo == MODE_SUMS, 0)) {
    // Reliable update, part 3: the sums of the next CG step for the true
    // residual r (now in memory with its halo) and the kept direction p:
    // r.z, z.Az, z.Ap and p.Ap, with z = D^-1 r on the tile's one-cell halo.
    float z[R + 2], zh[R], ph[R];
#pragma unroll
    for (int q = 0; q < R + 2; ++q)
      z[q] = ro[q + 1] * (JAC ? inv_diag(hy[q + 1], gy[q + 1], gy[q + 2], k.hx, k.gw, k.ge) : 1.f);
    const float zt = hr1 * (JAC ? inv_diag(hy_t, gs_t, gn_t, hx1, gw1, ge1) : 1.f);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      zh[q] = from_halo(zt, q + 1);
      ph[q] = from_halo(hp1, q + 1);
    }
    const auto rso = make_rsrc(rout, vbytes), pso = make_rsrc(pout, vbytes);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int j = j0 + q;
      float ze, zw, pe, pw;
      east_west(z[q + 1], zh[q], ze, zw);
      east_west(po[q + 2], ph[q], pe, pw);
      const float Az = stencil5(z[q + 1], ze, zw, z[q + 2], z[q], hy[q + 2], gy[q + 2], gy[q + 3], k.hx, k.gw, k.ge);
      const float sp = stencil5(po[q + 2], pe, pw, po[q + 3], po[q + 1], hy[q + 2], gy[q + 2], gy[q + 3], k.hx, k.gw,
                                k.ge);
      const uint32_t o = cell_off(ci.ok, j, ny, nx, ci.i);
      bstore(rso, o, ro[q + 2]);
      bstore(pso, o, po[q + 2]);
      // Off the grid every value and coefficient is 0, so the products are 0.
      acc[0] += (double)ro[q + 2] * (double)z[q + 1];
      acc[1] += (double)z[q + 1] * (double)Az;
      acc[2] += (double)z[q + 1] * (double)sp;
      acc[3] += (double)po[q + 2] * (double)sp;
      acc[4] += (double)ro[q + 2] * (double)ro[q + 2];
    }
    if (leader) {
      st->mode[par] = MODE_SUMS;
      st->it[par] = it;
      st->it_cg[par] = itcg;
      st->n_ru[par] = nru;
      st->rho[par] = gam_prev;
      st->rr_ru[par] = rr_ru;
      st->restart[par] = restart;
      st->dflag[par] = DONE_NO;
    }
  } else {
    // CG step. z and p on the own rows and, in the halo lanes, on the edge
    // and halo cells of this lane's row ...
    const float bet = (float)beta;
    const bool rst = beta == 0.0;
    float pv[R + 4], dv[R + 4];
#pragma unroll
    for (int q = 0; q < R + 4; ++q) {
      dv[q] = JAC ? inv_diag(hy[q], gy[q], gy[q + 1], k.hx, k.gw, k.ge) : 1.f;
      const float zv = ro[q] * dv[q];
      pv[q] = rst ? zv : zv + bet * po[q];
    }
    const float de = JAC ? inv_diag(hy_t, gs_t, gn_t, hxe, gwe, gee) : 1.f;
    const float d1 = JAC ? inv_diag(hy_t, gs_t, gn_t, hx1, gw1, ge1) : 1.f;
    const float d2 = JAC ? inv_diag(hy_t, gs_t, gn_t, hx2, gw2, ge2) : 1.f;
    const float pte = rst ? hre * de : hre * de + bet * hpe;
    const float pt1 = rst ? hr1 * d1 : hr1 * d1 + bet * hp1;
    const float pt2 = rst ? hr2 * d2 : hr2 * d2 + bet * hp2;
    // ... s = A p, r_{k+1} = r_k - alpha s and z_{k+1} on the halo column
    // (rows from the neighbouring lanes of the same side) ...
    const float alf = (float)alpha;
    const int pbits = __float_as_int(pt1);
    const float pt1n = __int_as_float(__builtin_amdgcn_update_dpp(0, pbits, 0x130, 0xf, 0xf, false));  // row + 1
    const float pt1s = __int_as_float(__builtin_amdgcn_update_dpp(0, pbits, 0x138, 0xf, 0xf, false));  // row - 1
    const float hve = ht.east ? pt2 : pte, hvw = ht.east ? pte : pt2;
    const float st1 = stencil5(pt1, hve, hvw, pt1n, pt1s, hy_t, gs_t, gn_t, hx1, gw1, ge1);
    const float zt1 = (hr1 - alf * st1) * d1;
    float p1h[R + 2], z1h[R];
#pragma unroll
    for (int q = 0; q < R + 2; ++q) p1h[q] = from_halo(pt1, q);
#pragma unroll
    for (int q = 0; q < R; ++q) z1h[q] = from_halo(zt1, q + 1);
    // ... and on the own rows j0-1 .. j0+R ...
    float sv[R + 2], rn[R + 2], zn[R + 2];
#pragma unroll
    for (int q = 0; q < R + 2; ++q) {  // own column, row j0-1+q
      float pe, pw;
      east_west(pv[q + 1], p1h[q], pe, pw);
      sv[q] = stencil5(pv[q + 1], pe, pw, pv[q + 2], pv[q], hy[q + 1], gy[q + 1], gy[q + 2], k.hx, k.gw, k.ge);
      rn[q] = ro[q + 1] - alf * sv[q];
      zn[q] = rn[q] * dv[q + 1];
    }
    // ... then A z_{k+1} on the tile, the stores and the sums.
    const auto rso = make_rsrc(rout, vbytes), pso = make_rsrc(pout, vbytes), xso = make_rsrc(xc, vbytes);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int j = j0 + q;
      float ze, zw;
      east_west(zn[q + 1], z1h[q], ze, zw);
      const float Az = stencil5(zn[q + 1], ze, zw, zn[q + 2], zn[q], hy[q + 2], gy[q + 2], gy[q + 3], k.hx, k.gw,
                                k.ge);
      const float pk = pv[q + 2];
      const uint32_t o = cell_off(ci.ok, j, ny, nx, ci.i);
      bstore(rso, o, rn[q + 1]);
      bstore(pso, o, pk);
      bstore(xso, o, xcv[q] + alf * pk);
      // Off the grid every value and coefficient is 0, so the products are 0.
      acc[0] += (double)rn[q + 1] * (double)zn[q + 1];
      acc[1] += (double)zn[q + 1] * (double)Az;
      acc[2] += (double)zn[q + 1] * (double)sv[q + 1];
      acc[3] += (double)pk * (double)sv[q + 1];
      acc[4] += (double)rn[q + 1] * (double)rn[q + 1];
    }
  }
  store_sums<kSums>(acc, lds, sums_of(a, par, s, nbs), P, blk);
}

template <int R, bool JAC>
__global__ __launch_bounds__(kBlock) void k_pcg1(PcgArgs a, int par) {
  __shared__ double lds[kSums * kWaves];
  pcg1_body<R, JAC>(a, blockIdx.z, gridDim.z, blockIdx.x, par, lds);
}

// Solves on grids of different sizes in one launch: work[b] = (solve << 20) |
// (workgroup within the solve) for the launch's workgroup b; descs[solve] is
// that solve's argument block (one solve each).
template <int R, bool JAC>
__global__ __launch_bounds__(kBlock) void k_pcg1_multi(const PcgArgs* __restrict__ descs,
                                                       const uint32_t* __restrict__ work, int par) {
  __shared__ double lds[kSums * kWaves];
  const uint32_t wv = __builtin_amdgcn_readfirstlane(work[blockIdx.x]);
  pcg1_body<R, JAC>(descs[wv >> 20], 0, 1, (int)(wv & 0xFFFFFu), par, lds);
}

// Set-up after the right-hand side: zero x_c and both p buffers and leave the
// state as after a FLUSH of parity 0, so that the first launch (parity 1)
// computes the true residual of the initial guess with p = 0 and a restart.
__global__ __launch_bounds__(kBlock) void k_pcg1_init(PcgArgs a) {
  __shared__ double lds[kWaves];
  const int s = blockIdx.z, nx = a.c.nx, ny = a.c.ny;
  SolveState* st = a.st + s;
  const double bb = reduce_partials(a.partA + (size_t)s * a.P, a.P, lds);
  const bool bad = st->nonfinite;
  if (is_first_block()) {
    st->bnorm2 = bb;
    st->thr2 = a.tol_kind == 1 ? a.tol * a.tol : a.tol * a.tol * bb;
    st->mode[0] = MODE_FLUSH;
    st->restart[0] = 1;
    st->it[0] = 0;
    st->it_cg[0] = 0;
    st->n_ru[0] = 0;
    st->alpha[0] = 0.0;
    st->rho[0] = 0.0;
    st->rr_ru[0] = 0.0;
    st->rr_last[0] = 0.0;
    st->brk[0] = 0;
    st->n_dlsm = 0;
    st->n_rej = 0;
    st->done = bad ? DONE_NONFINITE : DONE_NO;
    st->dflag[0] = st->dflag[1] = bad ? DONE_NONFINITE : DONE_NO;
    st->it_final = 0;
    st->nru_final = 0;
    st->itcg_final = 0;
    st->rr_final = 0.0;
    st->t_start = wall_clock64();
    st->t_done = st->t_start;
    a.flags[s] = bad ? DONE_NONFINITE : DONE_NO;
  }
  const size_t off = (size_t)s * a.N;
  const TileXY tl = tile_xy(nx, ny, a.R);
  const int i = tl.valid ? tl.i0 + (threadIdx.x & (kWave - 1)) : nx;
  if (i < nx)
    for (int q = 0; q < a.R; ++q) {
      const int j = tl.j0 + q;
      if (j >= ny) break;
      const size_t kk = off + (size_t)j * nx + i;
      a.xc[kk] = 0.f;
      a.p0[kk] = 0.f;
      a.p1[kk] = 0.f;
    }
}

#define PPE1_DISPATCH(R, JAC, ...)                                                   \
  do {                                                                               \
    if (JAC) {                                                                       \
      switch (R) {                                                                   \
        case 2: { constexpr int RR = 2; constexpr bool JJ = true; __VA_ARGS__; } break;  \
        case 4: { constexpr int RR = 4; constexpr bool JJ = true; __VA_ARGS__; } break;  \
        case 8: { constexpr int RR = 8; constexpr bool JJ = true; __VA_ARGS__; } break;  \
        default: { constexpr int RR = 16; constexpr bool JJ = true; __VA_ARGS__; } break; \
      }                                                                              \
    } else {                                                                         \
      switch (R) {                                                                   \
        case 2: { constexpr int RR = 2; constexpr bool JJ = false; __VA_ARGS__; } break;  \
        case 4: { constexpr int RR = 4; constexpr bool JJ = false; __VA_ARGS__; } break;  \
        case 8: { constexpr int RR = 8; constexpr bool JJ = false; __VA_ARGS__; } break;  \
        default: { constexpr int RR = 16; constexpr bool JJ = false; __VA_ARGS__; } break; \
      }                                                                              \
    }                                                                                \
  } while (0)

void launch_pcg1_setup(const PcgArgs& a, int nb, hipStream_t s) {
  const dim3 g = stencil_grid(a.c, a.R, nb);
  launch_rhs(a, nb, s);
  k_pcg1_init<<<g, kBlock, 0, s>>>(a);
  launch_pcg1_step(a, nb, 1, s);
}

void launch_pcg1_step(const PcgArgs& a, int nb, int par, hipStream_t s) {
  const dim3 g = stencil_grid(a.c, a.R, nb);
  PPE1_DISPATCH(a.R, a.jacobi, k_pcg1<RR, JJ><<<g, kBlock, 0, s>>>(a, par));
}

void launch_pcg1_multi_step(const PcgArgs* descs, const uint32_t* work, int nblocks, int R, bool jacobi, int par,
                            hipStream_t s) {
  PPE1_DISPATCH(R, jacobi, k_pcg1_multi<RR, JJ><<<nblocks, kBlock, 0, s>>>(descs, work, par));
}

void launch_pcg1_init(const PcgArgs& a, int nb, hipStream_t s) {
  k_pcg1_init<<<stencil_grid(a.c, a.R, nb), kBlock, 0, s>>>(a);
}

void launch_pcg1_step_timed(const PcgArgs& a, int nb, int par, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const dim3 g = stencil_grid(a.c, a.R, nb);
  PPE1_DISPATCH(a.R, a.jacobi, hipExtLaunchKernelGGL(k_pcg1<RR, JJ>, g, dim3(kBlock), 0, s, e0, e1, 0, a, par));
}

}  // namespace ppe
