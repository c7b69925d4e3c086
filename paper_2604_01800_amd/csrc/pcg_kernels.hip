// Stencil and fused Jacobi-PCG kernels (HIP, gfx950).
//
// Operator: the finite-volume form of the pressure Poisson matrix of Eq. 10,
// matrix-free from 1D coefficient arrays (see Coef). PCG: the textbook
// preconditioned CG (Saad, Alg. 9.1) with D = diag(A), reorganised into two
// fused passes per iteration, each ending in a fixed-order FP64 grid reduction:
//
//   phase A: x_c += alpha_{k-1} p_{k-1}          (deferred solution update)
//            p_k  = D^-1 r_k + beta_k p_{k-1}    (p recomputed on the halo)
//            q    = A p_k, partial sums of p.q   -> writes p_k, x_c   (20 B/cell)
//   phase B: alpha_k = rho_k / p.q
//            r   -= alpha_k A p_k (q recomputed), partial sums of r.r, r.z
//                                                -> writes r          (12 B/cell)
//
// Vectors are FP32; products of FP32 values are exact in FP64 and every sum is
// FP64. The solution is accumulated in FP64 by reliable updates (residual
// replacement, Sleijpen & van der Vorst 1996): when the recursive residual has
// fallen by delta against the last true residual (or claims convergence, or
// the iteration limit is hit), phase A flushes x_c into the FP64 solution and
// phase B recomputes r = b - A x in FP64. Convergence is declared only on that
// FP64 true residual, with the L2 stopping rule of Sec. 2.2.
//
// Layout: one wavefront owns a 64-column strip and walks R rows down, keeping
// the rows above/below in registers; east/west neighbours come from lane
// shuffles, and lanes 0 and 63 load the halo columns. Workgroup = 4 waves =
// 64 x 4R cells. Each workgroup of the consuming kernel re-reduces the
// producer's per-workgroup partials in the same order, so all workgroups see
// bit-identical scalars and take identical decisions without atomics.
#include <hip/hip_ext.h>

#include "common.hpp"
#include "kernels.hpp"
#include "stencil.hpp"

namespace ppe {

// ---------------------------------------------------------------------------
// y = A x for a batch (parity checks and the line-search step).
template <typename T, int R, bool M>
__global__ __launch_bounds__(kBlock) void k_apply(Coef c, const T* __restrict__ x, T* __restrict__ y) {
  const int nx = c.nx, ny = c.ny;
  const size_t off = (size_t)blockIdx.z * nx * ny;
  x += off;
  y += off;
  const T* hx = sizeof(T) == 8 ? (const T*)c.hx64 : (const T*)c.hx;
  const T* hy = sizeof(T) == 8 ? (const T*)c.hy64 : (const T*)c.hy;
  const T* gx = sizeof(T) == 8 ? (const T*)c.gx64 : (const T*)c.gx;
  const T* gy = sizeof(T) == 8 ? (const T*)c.gy64 : (const T*)c.gy;
  const TileXY tl = tile_xy(nx, ny, R);
  if (!tl.valid) return;
  const ColCtx<T> cc = col_ctx<T>(nx, hx, gx, tl.i0);
  const int j0 = tl.j0;
  if (j0 >= ny) return;
  T vprev = (j0 > 0 && cc.ok) ? x[(size_t)(j0 - 1) * nx + cc.i] : T(0);
  T vcur = cc.ok ? x[(size_t)j0 * nx + cc.i] : T(0);
  // solid-mask operator: fluid flags of the same cells (0 off the grid)
  auto flag = [&](bool ok, int j, int i) { return (M && ok) ? (T)c.fl[(size_t)j * nx + i] : T(0); };
  T mprev = flag(j0 > 0 && cc.ok, j0 - 1, cc.i);
  T mcur = flag(cc.ok, j0, cc.i);
  for (int q = 0; q < R; ++q) {
    const int j = j0 + q;
    if (j >= ny) break;
    const T vnext = (j + 1 < ny && cc.ok) ? x[(size_t)(j + 1) * nx + cc.i] : T(0);
    const T vh = cc.hok ? x[(size_t)j * nx + cc.ih] : T(0);
    T ve, vw;
    east_west(vcur, vh, ve, vw);
    T v;
    if (M) {
      const T mnext = flag(j + 1 < ny && cc.ok, j + 1, cc.i);
      const T mh = flag(cc.hok, j, cc.ih);
      T me, mw;
      east_west(mcur, mh, me, mw);
      const T sum = hy[j] * (cc.ge * me * (vcur - ve) + cc.gw * mw * (vcur - vw)) +
                    cc.hx * (gy[j + 1] * mnext * (vcur - vnext) + gy[j] * mprev * (vcur - vprev));
      v = mcur * sum + (T(1) - mcur) * vcur;
      mprev = mcur;
      mcur = mnext;
    } else {
      v = stencil5(vcur, ve, vw, vnext, vprev, hy[j], gy[j], gy[j + 1], cc.hx, cc.gw, cc.ge);
    }
    if (cc.ok) y[(size_t)j * nx + cc.i] = v;
    vprev = vcur;
    vcur = vnext;
  }
}

// ---------------------------------------------------------------------------
// Right-hand side: b = (cell area) f - mean. Pass 1: partial sums of area*f
// and a count of non-finite source values.
__global__ __launch_bounds__(kBlock) void k_rhs_sum(PcgArgs a) {
  __shared__ double lds[kWaves];
  const int s = blockIdx.z, nx = a.c.nx, ny = a.c.ny;
  const float* f = a.call->f + (size_t)s * a.N;
  const TileXY tl = tile_xy(nx, ny, a.R);
  const int i = tl.valid ? tl.i0 + (threadIdx.x & (kWave - 1)) : nx;
  const int j0 = tl.j0;
  double sum = 0.0, bad = 0.0;
  if (i < nx) {
    const double hxi = a.c.hx64[i];
    for (int q = 0; q < a.R; ++q) {
      const int j = j0 + q;
      if (j >= ny) break;
      const float v = f[(size_t)j * nx + i];
      if (!isfinite(v)) bad += 1.0;
      else if (!a.c.fl || a.c.fl[(size_t)j * nx + i] != 0.f) sum += hxi * a.c.hy64[j] * (double)v;
    }
  }
  sum = block_sum(sum, lds);
  bad = block_sum(bad, lds);
  if (threadIdx.x == 0) {
    double* pb = a.partB + (size_t)s * 2 * a.P;
    pb[block_linear()] = sum;
    pb[a.P + block_linear()] = bad;
  }
}

// Pass 2: the mean, then partial sums of |b|^2.
__global__ __launch_bounds__(kBlock) void k_rhs_norm(PcgArgs a) {
  __shared__ double lds[kWaves];
  const int s = blockIdx.z, nx = a.c.nx, ny = a.c.ny;
  const double* pb = a.partB + (size_t)s * 2 * a.P;
  const double sum = reduce_partials(pb, a.P, lds);
  const double bad = reduce_partials(pb + a.P, a.P, lds);
  // the mean over the cells of the operator (the fluid cells with a solid mask)
  const double mean = sum / (double)(a.c.fl ? a.c.nfluid : a.N);
  SolveState* st = a.st + s;
  if (is_first_block()) {
    st->bmean = mean;
    st->nonfinite = bad > 0.0;
  }
  const float* f = a.call->f + (size_t)s * a.N;
  const TileXY tl = tile_xy(nx, ny, a.R);
  const int i = tl.valid ? tl.i0 + (threadIdx.x & (kWave - 1)) : nx;
  const int j0 = tl.j0;
  double bb = 0.0;
  if (i < nx && bad == 0.0) {
    const double hxi = a.c.hx64[i];
    for (int q = 0; q < a.R; ++q) {
      const int j = j0 + q;
      if (j >= ny) break;
      const double b = (a.c.fl && a.c.fl[(size_t)j * nx + i] == 0.f)
                           ? 0.0
                           : hxi * a.c.hy64[j] * (double)f[(size_t)j * nx + i] - mean;
      bb += b * b;
    }
  }
  if (a.zero_x0 && i < nx) {
    double* x = a.call->x + (size_t)s * a.N;
    for (int q = 0; q < a.R; ++q) {
      const int j = j0 + q;
      if (j >= ny) break;
      x[(size_t)j * nx + i] = 0.0;
    }
  }
  bb = block_sum(bb, lds);
  if (threadIdx.x == 0) a.partA[(size_t)s * a.P + block_linear()] = bb;
}

// True residual r = b - A x in FP64 over this wave's rows; stores r in FP32
// and accumulates |r|^2 (FP64 value) and r.D^-1 r (FP32 value, exact products).
// It runs a handful of times per solve, so it walks the rows with a small
// register footprint instead of holding a full FP64 tile.
// Preconditioner variants of the two-phase kernels: PC 0 none, 1 Jacobi,
// 2 a supplied z (multigrid); 3 and 4 are 0 and 1 on the solid-mask operator.
template <int PC>
struct PcKind {
  static constexpr bool mask = PC >= 3;
  static constexpr int base = PC >= 3 ? PC - 3 : PC;
};

template <int R, int PC>
__device__ __forceinline__ void true_residual_rows(const PcgArgs& a, int s, double& acc_rr, double& acc_rz) {
  constexpr bool M = PcKind<PC>::mask;
  constexpr int PB = PcKind<PC>::base;
  const int nx = a.c.nx, ny = a.c.ny;
  const size_t off = (size_t)s * a.N;
  const double* __restrict__ x = a.call->x + off;
  const float* __restrict__ f = a.call->f + off;
  float* __restrict__ r = a.r + off;
  const TileXY tl = tile_xy(nx, ny, R);
  const ColIdx ci = col_idx(nx, tl);
  const int j0 = tl.j0;
  if (j0 >= ny) return;
  const ColCoef<double> k = load_cols<double>(a.c.hx64, a.c.gx64, ci);
  const ColCoef<float> kf = load_cols<float>(a.c.hx, a.c.gx, ci);
  const double bmean = a.st[s].bmean;
  double vprev = (ci.ok && j0 > 0) ? x[(size_t)(j0 - 1) * nx + ci.i] : 0.0;
  double vcur = ci.ok ? x[(size_t)j0 * nx + ci.i] : 0.0;
  auto flag = [&](bool ok, int j, int i) { return (M && ok) ? (double)a.c.fl[(size_t)j * nx + i] : 0.0; };
  double mprev = flag(ci.ok && j0 > 0, j0 - 1, ci.i);
  double mcur = flag(ci.ok, j0, ci.i);
#pragma unroll 1
  for (int q = 0; q < R; ++q) {
    const int j = j0 + q;
    if (j >= ny) break;
    const double vnext = (ci.ok && j + 1 < ny) ? x[(size_t)(j + 1) * nx + ci.i] : 0.0;
    const double vh = ci.hok ? x[(size_t)j * nx + ci.ih] : 0.0;
    const float fv = ci.ok ? f[(size_t)j * nx + ci.i] : 0.f;
    double ve, vw;
    east_west(vcur, vh, ve, vw);
    const double hyj = a.c.hy64[j];
    double Ax, bv;
    if (M) {
      const double mnext = flag(ci.ok && j + 1 < ny, j + 1, ci.i);
      const double mh = flag(ci.hok, j, ci.ih);
      double me, mw;
      east_west(mcur, mh, me, mw);
      const double sum = hyj * (k.ge * me * (vcur - ve) + k.gw * mw * (vcur - vw)) +
                         k.hx * (a.c.gy64[j + 1] * mnext * (vcur - vnext) + a.c.gy64[j] * mprev * (vcur - vprev));
      Ax = mcur * sum + (1.0 - mcur) * vcur;
      bv = mcur * (k.hx * hyj * (double)fv - bmean);
      mprev = mcur;
      mcur = mnext;
    } else {
      Ax = stencil5(vcur, ve, vw, vnext, vprev, hyj, a.c.gy64[j], a.c.gy64[j + 1], k.hx, k.gw, k.ge);
      bv = k.hx * hyj * (double)fv - bmean;
    }
    if (ci.ok) {
      const double rv = bv - Ax;
      const float rr = (float)rv;
      r[(size_t)j * nx + ci.i] = rr;
      acc_rr += rv * rv;
      if (PB != 2) {
        float z = rr;
        if (PB == 1)
          z = M ? rr * a.c.dinv[(size_t)j * nx + ci.i]
                : rr / (a.c.hy[j] * (kf.gw + kf.ge) + kf.hx * (a.c.gy[j] + a.c.gy[j + 1]));
        acc_rz += (double)rr * (double)z;
      }
    }
    vprev = vcur;
    vcur = vnext;
  }
}

template <int R, int PC>
__global__ __launch_bounds__(kBlock) void k_pcg_init(PcgArgs a) {
  __shared__ double lds[kWaves];
  const int s = blockIdx.z, nx = a.c.nx, ny = a.c.ny;
  SolveState* st = a.st + s;
  const double bb = reduce_partials(a.partA + (size_t)s * a.P, a.P, lds);
  const bool bad = st->nonfinite;
  if (is_first_block()) {
    st->bnorm2 = bb;
    st->thr2 = a.tol_kind == 1 ? a.tol * a.tol : a.tol * a.tol * bb;
    st->mode[1] = MODE_TRUE;
    st->restart[1] = 1;
    st->it[1] = 0;
    st->it_cg[1] = 0;
    st->n_ru[1] = 0;
    st->alpha[1] = 0.0;
    st->rho[1] = 0.0;
    st->rr_ru[1] = 0.0;
    st->rr_last[1] = 0.0;
    st->brk[1] = 0;
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
    st->t_mark = st->t_start;
    st->t_acc[0] = st->t_acc[1] = st->t_acc[2] = 0;
    a.flags[s] = bad ? DONE_NONFINITE : DONE_NO;
  }
  double rr = 0.0, rz = 0.0;
  if (!bad) {
    const size_t off = (size_t)s * a.N;
    const TileXY tl = tile_xy(nx, ny, R);
    const int i = tl.valid ? tl.i0 + (threadIdx.x & (kWave - 1)) : nx;
    const int j0 = tl.j0;
    if (i < nx) {
      for (int q = 0; q < R; ++q) {
        const int j = j0 + q;
        if (j >= ny) break;
        const size_t k = off + (size_t)j * nx + i;
        a.xc[k] = 0.f;
        a.p0[k] = 0.f;
        a.p1[k] = 0.f;
      }
    }
    true_residual_rows<R, PC>(a, s, rr, rz);
  }
  rr = block_sum(rr, lds);
  rz = block_sum(rz, lds);
  if (threadIdx.x == 0) {
    double* pb = a.partB + (size_t)s * 2 * a.P;
    pb[block_linear()] = rr;
    pb[a.P + block_linear()] = rz;
  }
}

// ---------------------------------------------------------------------------
// Phase A. par selects the p buffer written (p[par]) and the state slots.
// force != 0 makes this pass a reliable update (used after line-search
// blocks); force_restart then also restarts CG (beta = 0) afterwards.
template <int R, int PC>
__global__ __launch_bounds__(kBlock) void k_pcg_a(PcgArgs a, int par, int force, int force_restart) {
  constexpr bool M = PcKind<PC>::mask;
  constexpr int PB = PcKind<PC>::base;
  __shared__ double lds[kWaves];
  const int s = blockIdx.z, nx = a.c.nx, ny = a.c.ny;
  SolveState* st = a.st + s;
  const int P = a.P, pm = par ^ 1;
  const size_t off = (size_t)s * a.N;
  const float* __restrict__ r = a.r + off;
  float* __restrict__ xc = a.xc + off;
  const float* __restrict__ pold = (par ? a.p0 : a.p1) + off;
  float* __restrict__ pnew = (par ? a.p1 : a.p0) + off;
  const TileXY tl = tile_xy(nx, ny, R);
  const ColIdx ci = col_idx(nx, tl);
  const int j0 = tl.j0;

  // Tile loads first: they do not depend on the scalars reduced below.
  const uint64_t vbytes = (uint64_t)a.N * 4;
  Tile<float, R> tr, tp;
  float xcv[R];
  // the preconditioned residual: D^-1 r formed below, or z = M^-1 r supplied (PC = 2)
  load_tile<R>(make_rsrc(PB == 2 ? a.z + off : r, vbytes), nx, ny, j0, ci, tr);
  load_tile<R>(make_rsrc(pold, vbytes), nx, ny, j0, ci, tp);
  // solid-mask operator: fluid flags and the inverse diagonal on the tile
  Tile<float, R> tm, td;
  if (M) {
    load_tile<R>(make_rsrc(a.c.fl, vbytes), nx, ny, j0, ci, tm);
    if (PB == 1) load_tile<R>(make_rsrc(a.c.dinv, vbytes), nx, ny, j0, ci, td);
  }
  load_rows_own<R>(make_rsrc(xc, vbytes), nx, ny, j0, ci, xcv);
  RowCoef<float, R> rc;
  load_rows<float, R>(a.c.hy, a.c.gy, j0, rc);
  const ColCoef<float> k = load_cols<float>(a.c.hx, a.c.gx, ci);

  // State of the previous launches (never written by this launch).
  const int dprev = st->dflag[pm];
  const int max_iter = a.call->max_iter;
  const double delta2 = a.call->delta2;
  const int prev_mode = st->mode[pm];
  const int it = st->it[pm], nru = st->n_ru[pm], itcg = st->it_cg[pm];
  const int restart = st->restart[pm], brk = st->brk[pm];
  const double rho_prev = st->rho[pm], alpha_pm = st->alpha[pm], thr2 = st->thr2;
  double rr_ru = st->rr_ru[pm];
  const bool leader = is_first_block();
  // The partial sums are reduced before the done test so that the tile loads
  // above are already in flight whichever way the test goes.
  const double* pb = a.partB + (size_t)s * 2 * P;
  const double rr = reduce_partials(pb, P, lds);
  const double rz = reduce_partials(pb + P, P, lds);
  if (dprev) {
    if (leader) st->dflag[par] = dprev;
    return;
  }
  // residual history: the norm after `it` iterations (the recursive residual,
  // or the true one after a reliable update, which overwrites it)
  if (leader && a.hist && it < a.hist_cap) {
    const double bb = st->bnorm2;
    a.hist[(size_t)s * a.hist_cap + it] = bb > 0.0 ? sqrt(rr / bb) : sqrt(rr);
  }
  int done = DONE_NO;
  bool flush = false;
  if (prev_mode == MODE_TRUE) {
    // The last phase B computed the FP64 true residual: judge convergence.
    rr_ru = rr;
    if (!isfinite(rr)) done = DONE_NONFINITE;
    else if (rr <= thr2) done = DONE_CONV;
    else if (it >= max_iter) done = DONE_MAXIT;
    flush = force;
  } else {
    flush = force || brk || !isfinite(rr) || rr <= thr2 || rr <= delta2 * rr_ru || it >= max_iter;
  }
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

  if (flush) {
    // Reliable update, part 1: x += x_c + alpha p_old in FP64; x_c = 0; p carried over.
    double* __restrict__ x = a.call->x + off;
    const double al = alpha_pm;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int j = j0 + q;
      if (ci.ok && j < ny) {
        const size_t kk = (size_t)j * nx + ci.i;
        const float po = tp.own[q + 1];
        x[kk] = x[kk] + ((double)xcv[q] + al * (double)po);
        xc[kk] = 0.f;
        pnew[kk] = po;
      }
    }
    if (leader) {
      st->dflag[par] = DONE_NO;
      st->mode[par] = MODE_TRUE;
      st->it[par] = it;
      st->it_cg[par] = itcg;
      st->n_ru[par] = nru + 1;
      st->rho[par] = rho_prev;
      st->rr_ru[par] = rr_ru;
      st->rr_last[par] = rr;
      st->restart[par] = (force && force_restart) || brk;
      st->brk[par] = 0;
    }
    return;
  }

  double beta_d = (prev_mode == MODE_TRUE && restart) ? 0.0 : rz / rho_prev;
  if (!isfinite(beta_d)) beta_d = 0.0;
  const float beta = (float)beta_d;
  const float alpha_prev = (float)alpha_pm;
  // p = D^-1 r + beta p_old on the own rows (j0-1 .. j0+R) and the halo rows.
  // Off the grid r = p_old = 0 and the diagonal is 0; the fmax keeps 0/0 out.
  Tile<float, R> pn;
#pragma unroll
  for (int q = 0; q < R + 2; ++q) {
    float z = tr.own[q];
    if (PB == 1) {
      if (M) z = z * td.own[q];
      else z = z / fmaxf(rc.hy[q] * (k.gw + k.ge) + k.hx * (rc.gy[q] + rc.gy[q + 1]), 1e-30f);
    }
    pn.own[q] = z + beta * tp.own[q];
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    float z = tr.halo[q];
    if (PB == 1) {
      if (M) z = z * td.halo[q];
      else z = z / fmaxf(rc.hy[q + 1] * (k.gwh + k.geh) + k.hxh * (rc.gy[q + 1] + rc.gy[q + 2]), 1e-30f);
    }
    pn.halo[q] = z + beta * tp.halo[q];
  }
  float Ap[R];
  if (M) stencil_rows_masked<R>(pn, tm, rc, k, Ap);
  else stencil_rows<float, R>(pn, rc, k, Ap);
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int j = j0 + q;
    if (ci.ok && j < ny) {
      const size_t kk = (size_t)j * nx + ci.i;
      const float pv = pn.own[q + 1];
      pnew[kk] = pv;
      xc[kk] = xcv[q] + alpha_prev * tp.own[q + 1];
      acc += (double)pv * (double)Ap[q];
    }
  }
  acc = block_sum(acc, lds);
  if (threadIdx.x == 0) a.partA[(size_t)s * P + block_linear()] = acc;
  if (leader) {
    st->dflag[par] = DONE_NO;
    st->mode[par] = MODE_CG;
    st->it[par] = it + 1;
    st->it_cg[par] = itcg + 1;
    st->n_ru[par] = nru;
    st->rho[par] = rz;
    st->rr_ru[par] = rr_ru;
    st->rr_last[par] = rr;
    st->restart[par] = 0;
    st->brk[par] = 0;
  }
}

// Phase B: CG residual update, or the FP64 true residual after a flush.
template <int R, int PC>
__global__ __launch_bounds__(kBlock) void k_pcg_b(PcgArgs a, int par) {
  constexpr bool M = PcKind<PC>::mask;
  constexpr int PB = PcKind<PC>::base;
  __shared__ double lds[kWaves];
  const int s = blockIdx.z, nx = a.c.nx, ny = a.c.ny;
  SolveState* st = a.st + s;
  const int dprev = st->dflag[par];  // written by the phase A before this launch
  const int mode = st->mode[par];
  const int P = a.P;
  const bool leader = is_first_block();
  double acc_rr = 0.0, acc_rz = 0.0;
  if (mode == MODE_TRUE) {
    if (dprev) return;
    true_residual_rows<R, PC>(a, s, acc_rr, acc_rz);
    if (leader) {
      st->alpha[par] = 0.0;
      st->brk[par] = 0;
    }
  } else {
    const size_t off = (size_t)s * a.N;
    float* __restrict__ r = a.r + off;
    const float* __restrict__ p = (par ? a.p1 : a.p0) + off;
    const TileXY tl = tile_xy(nx, ny, R);
    const ColIdx ci = col_idx(nx, tl);
    const int j0 = tl.j0;
    const uint64_t vbytes = (uint64_t)a.N * 4;
    Tile<float, R> tp, tm;
    float rv[R], dv[R];
    load_tile<R>(make_rsrc(p, vbytes), nx, ny, j0, ci, tp);
    load_rows_own<R>(make_rsrc(r, vbytes), nx, ny, j0, ci, rv);
    if (M) {
      load_tile<R>(make_rsrc(a.c.fl, vbytes), nx, ny, j0, ci, tm);
      if (PB == 1) load_rows_own<R>(make_rsrc(a.c.dinv, vbytes), nx, ny, j0, ci, dv);
    }
    RowCoef<float, R> rc;
    load_rows<float, R>(a.c.hy, a.c.gy, j0, rc);
    const ColCoef<float> k = load_cols<float>(a.c.hx, a.c.gx, ci);
    const double rho = st->rho[par];
    const double pq = reduce_partials(a.partA + (size_t)s * P, P, lds);
    if (dprev) return;
    double al = rho / pq;
    const bool brk = !(pq > 0.0) || !isfinite(al);
    if (brk) al = 0.0;
    const float alf = (float)al;
    float Ap[R];
    if (M) stencil_rows_masked<R>(tp, tm, rc, k, Ap);
    else stencil_rows<float, R>(tp, rc, k, Ap);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int j = j0 + q;
      if (ci.ok && j < ny) {
        const float rn = rv[q] - alf * Ap[q];
        r[(size_t)j * nx + ci.i] = rn;
        acc_rr += (double)rn * (double)rn;
        if (PB != 2) {
          float z = rn;
          if (PB == 1) z = M ? rn * dv[q] : rn / (rc.hy[q + 1] * (k.gw + k.ge) + k.hx * (rc.gy[q + 1] + rc.gy[q + 2]));
          acc_rz += (double)rn * (double)z;
        }
      }
    }
    if (leader) {
      st->alpha[par] = al;
      st->brk[par] = brk;
    }
  }
  acc_rr = block_sum(acc_rr, lds);
  acc_rz = block_sum(acc_rz, lds);
  if (threadIdx.x == 0) {
    double* pb = a.partB + (size_t)s * 2 * P;
    pb[block_linear()] = acc_rr;
    pb[P + block_linear()] = acc_rz;
  }
}

// ---------------------------------------------------------------------------
// Line-search step of the hybrid solve (Eqs. 12-13) along a direction e:
//   alpha = r.e / e.Ae,  x += alpha e,  r -= alpha A e.
// Kernel 1 forms the partial sums r.e, e.Ae, e.e; kernel 2 reduces them,
// applies the guard (reject when e.Ae <= 1e-30 e.e or a value is not finite:
// the step is skipped and counted, PCG continues) and updates x_c and r,
// recomputing A e. par is the parity of the last CG phase-A launch, whose
// state slots hold the done flag and the iteration count.
template <int R>
__global__ __launch_bounds__(kBlock) void k_dlsm_a(PcgArgs a, int par) {
  __shared__ double lds[kWaves];
  const int s = blockIdx.z, nx = a.c.nx, ny = a.c.ny;
  SolveState* st = a.st + s;
  const int dprev = st->dflag[par];
  const int it = st->it[par];
  const int active = !dprev && it < a.call->max_iter;
  if (is_first_block()) {
    st->dl_active = active;
    st->dl_it = it + active;
  }
  if (!active) return;
  const size_t off = (size_t)s * a.N;
  const uint64_t vbytes = (uint64_t)a.N * 4;
  const TileXY tl = tile_xy(nx, ny, R);
  const ColIdx ci = col_idx(nx, tl);
  const int j0 = tl.j0;
  Tile<float, R> te;
  float rv[R];
  load_tile<R>(make_rsrc(a.e + off, vbytes), nx, ny, j0, ci, te);
  load_rows_own<R>(make_rsrc(a.r + off, vbytes), nx, ny, j0, ci, rv);
  RowCoef<float, R> rc;
  load_rows<float, R>(a.c.hy, a.c.gy, j0, rc);
  const ColCoef<float> k = load_cols<float>(a.c.hx, a.c.gx, ci);
  float Ae[R];
  stencil_rows<float, R>(te, rc, k, Ae);
  double num = 0.0, den = 0.0, ee = 0.0;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    if (ci.ok && j0 + q < ny) {
      const double ev = te.own[q + 1];
      num += (double)rv[q] * ev;
      den += ev * (double)Ae[q];
      ee += ev * ev;
    }
  }
  num = block_sum(num, lds);
  den = block_sum(den, lds);
  ee = block_sum(ee, lds);
  if (threadIdx.x == 0) {
    double* pd = a.partD + (size_t)s * 3 * a.P;
    pd[block_linear()] = num;
    pd[a.P + block_linear()] = den;
    pd[2 * a.P + block_linear()] = ee;
  }
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_dlsm_b(PcgArgs a, int par) {
  __shared__ double lds[kWaves];
  const int s = blockIdx.z, nx = a.c.nx, ny = a.c.ny;
  SolveState* st = a.st + s;
  const int active = st->dl_active;
  const int itn = st->dl_it;
  const bool leader = is_first_block();
  if (!active) return;
  const size_t off = (size_t)s * a.N;
  const uint64_t vbytes = (uint64_t)a.N * 4;
  const TileXY tl = tile_xy(nx, ny, R);
  const ColIdx ci = col_idx(nx, tl);
  const int j0 = tl.j0;
  float* __restrict__ r = a.r + off;
  float* __restrict__ xc = a.xc + off;
  Tile<float, R> te;
  float rv[R], xv[R];
  load_tile<R>(make_rsrc(a.e + off, vbytes), nx, ny, j0, ci, te);
  load_rows_own<R>(make_rsrc(r, vbytes), nx, ny, j0, ci, rv);
  load_rows_own<R>(make_rsrc(xc, vbytes), nx, ny, j0, ci, xv);
  RowCoef<float, R> rc;
  load_rows<float, R>(a.c.hy, a.c.gy, j0, rc);
  const ColCoef<float> k = load_cols<float>(a.c.hx, a.c.gx, ci);
  const double* pd = a.partD + (size_t)s * 3 * a.P;
  const double num = reduce_partials(pd, a.P, lds);
  const double den = reduce_partials(pd + a.P, a.P, lds);
  const double ee = reduce_partials(pd + 2 * a.P, a.P, lds);
  const double alpha = num / den;
  const bool ok = isfinite(num) && isfinite(den) && isfinite(alpha) && den > 1e-30 * ee;
  if (leader) {
    st->it[par] = itn;
    st->dl_alpha = ok ? alpha : 0.0;
    if (ok) {
      st->n_dlsm += 1;
      st->mode[par] = MODE_CG;  // r and x_c changed: the next pass must recompute the true residual
    } else {
      st->n_rej += 1;
    }
  }
  double rr = 0.0;
  if (!ok) {
    // rejected: r is unchanged; its norm only matters for the history
    if (a.hist) {
#pragma unroll
      for (int q = 0; q < R; ++q)
        if (ci.ok && j0 + q < ny) rr += (double)rv[q] * (double)rv[q];
      rr = block_sum(rr, lds);
      if (threadIdx.x == 0) a.partA[(size_t)s * a.P + block_linear()] = rr;
    }
    return;
  }
  const float af = (float)alpha;
  float Ae[R];
  stencil_rows<float, R>(te, rc, k, Ae);
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int j = j0 + q;
    if (ci.ok && j < ny) {
      const size_t kk = (size_t)j * nx + ci.i;
      xc[kk] = xv[q] + af * te.own[q + 1];
      const float rn = rv[q] - af * Ae[q];
      r[kk] = rn;
      rr += (double)rn * (double)rn;
    }
  }
  // the partial sums of |r|^2 for the history (phase A's slots are free
  // during a line-search block: the next phase A rewrites them)
  if (a.hist) {
    rr = block_sum(rr, lds);
    if (threadIdx.x == 0) a.partA[(size_t)s * a.P + block_linear()] = rr;
  }
}

// History entry after a line-search step: |r| / |b| at the step's iteration
// count. One workgroup per solve.
__global__ __launch_bounds__(kBlock) void k_hist_dlsm(PcgArgs a) {
  __shared__ double lds[kWaves];
  const int s = blockIdx.z;
  SolveState* st = a.st + s;
  if (!st->dl_active) return;
  const double rr = reduce_partials(a.partA + (size_t)s * a.P, a.P, lds);
  const int it = st->dl_it;
  if (threadIdx.x == 0 && it < a.hist_cap) {
    const double bb = st->bnorm2;
    a.hist[(size_t)s * a.hist_cap + it] = bb > 0.0 ? sqrt(rr / bb) : sqrt(rr);
  }
}

// History entry after a block of CG iterations (before a line-search
// block): the residual the last phase B left, at the iteration count its
// phase A recorded in slot par. One workgroup per solve.
__global__ __launch_bounds__(kBlock) void k_hist_cg(PcgArgs a, int par) {
  __shared__ double lds[kWaves];
  const int s = blockIdx.z;
  SolveState* st = a.st + s;
  if (st->dflag[par]) return;
  const double rr = reduce_partials(a.partB + (size_t)s * 2 * a.P, a.P, lds);
  const int it = st->it[par];
  if (threadIdx.x == 0 && it < a.hist_cap) {
    const double bb = st->bnorm2;
    a.hist[(size_t)s * a.hist_cap + it] = bb > 0.0 ? sqrt(rr / bb) : sqrt(rr);
  }
}

// Phase clock of the hybrid solve: adds the time since the last mark to
// phase `cat` (0 CG-type, 1 network, 2 line search; -1 only marks), unless
// every solve of the call has decided. One thread.
__global__ void k_mark(PcgArgs a, int nb, int cat) {
  bool all = true;
  for (int s = 0; s < nb; ++s) all = all && a.flags[s] != DONE_NO;
  if (all) return;
  const uint64_t t = wall_clock64();
  SolveState* st = a.st;
  if (cat >= 0) st->t_acc[cat] += t - st->t_mark;
  st->t_mark = t;
}

// Test directions that replace the network: 1 zero, 2 Jacobi D^-1 r, 3 NaN, 4 ones.
template <int R>
__global__ __launch_bounds__(kBlock) void k_direction(PcgArgs a, int mode, float* __restrict__ e) {
  const int s = blockIdx.z, nx = a.c.nx, ny = a.c.ny;
  const size_t off = (size_t)s * a.N;
  const TileXY tl = tile_xy(nx, ny, R);
  const ColIdx ci = col_idx(nx, tl);
  const int j0 = tl.j0;
  const ColCoef<float> k = load_cols<float>(a.c.hx, a.c.gx, ci);
  for (int q = 0; q < R; ++q) {
    const int j = j0 + q;
    if (!ci.ok || j >= ny) continue;
    const size_t kk = off + (size_t)j * nx + ci.i;
    float v = 0.f;
    if (mode == 2) v = a.r[kk] / (a.c.hy[j] * (k.gw + k.ge) + k.hx * (a.c.gy[j] + a.c.gy[j + 1]));
    else if (mode == 3) v = __builtin_nanf("");
    else if (mode == 4) v = 1.f;
    e[kk] = v;
  }
}

// y = A x for nb samples on their own grids of one size (coefs[s] per sample).
template <int R>
__global__ __launch_bounds__(kBlock) void k_apply_multi(const Coef* __restrict__ coefs, const float* __restrict__ x,
                                                        float* __restrict__ y) {
  const Coef c = coefs[blockIdx.z];
  const int nx = c.nx, ny = c.ny;
  const size_t off = (size_t)blockIdx.z * nx * ny;
  const uint64_t vbytes = (uint64_t)nx * ny * 4;
  const TileXY tl = tile_xy(nx, ny, R);
  const ColIdx ci = col_idx(nx, tl);
  const int j0 = tl.j0;
  Tile<float, R> tv;
  load_tile<R>(make_rsrc(x + off, vbytes), nx, ny, j0, ci, tv);
  RowCoef<float, R> rc;
  load_rows<float, R>(c.hy, c.gy, j0, rc);
  const ColCoef<float> k = load_cols<float>(c.hx, c.gx, ci);
  float Av[R];
  stencil_rows<float, R>(tv, rc, k, Av);
#pragma unroll
  for (int q = 0; q < R; ++q)
    if (ci.ok && j0 + q < ny) y[off + (size_t)(j0 + q) * nx + ci.i] = Av[q];
}

void launch_apply_multi(const Coef* coefs, int nx, int ny, int nb, const float* x, float* y, hipStream_t s) {
  Coef c{};
  c.nx = nx;
  c.ny = ny;
  const dim3 g = stencil_grid(c, 4, nb);
  k_apply_multi<4><<<g, kBlock, 0, s>>>(coefs, x, y);
}

// Minimum-norm output: subtract the plain mean of x.
__global__ __launch_bounds__(kBlock) void k_x_sum(PcgArgs a) {
  __shared__ double lds[kWaves];
  const int s = blockIdx.z, nx = a.c.nx, ny = a.c.ny;
  const double* x = a.call->x + (size_t)s * a.N;
  const TileXY tl = tile_xy(nx, ny, a.R);
  const int i = tl.valid ? tl.i0 + (threadIdx.x & (kWave - 1)) : nx;
  const int j0 = tl.j0;
  double sum = 0.0;
  if (i < nx)
    for (int q = 0; q < a.R; ++q) {
      const int j = j0 + q;
      if (j >= ny) break;
      if (!a.c.fl || a.c.fl[(size_t)j * nx + i] != 0.f) sum += x[(size_t)j * nx + i];
    }
  sum = block_sum(sum, lds);
  if (threadIdx.x == 0) a.partA[(size_t)s * a.P + block_linear()] = sum;
}

__global__ __launch_bounds__(kBlock) void k_x_shift(PcgArgs a) {
  __shared__ double lds[kWaves];
  const int s = blockIdx.z, nx = a.c.nx, ny = a.c.ny;
  // the minimum-norm solution: zero mean over the operator's cells (the
  // fluid cells with a solid mask, whose solid cells keep their values)
  const double mean = reduce_partials(a.partA + (size_t)s * a.P, a.P, lds) / (double)(a.c.fl ? a.c.nfluid : a.N);
  if (is_first_block()) a.st[s].xmean = mean;
  double* x = a.call->x + (size_t)s * a.N;
  const TileXY tl = tile_xy(nx, ny, a.R);
  const int i = tl.valid ? tl.i0 + (threadIdx.x & (kWave - 1)) : nx;
  const int j0 = tl.j0;
  if (i < nx)
    for (int q = 0; q < a.R; ++q) {
      const int j = j0 + q;
      if (j >= ny) break;
      if (!a.c.fl || a.c.fl[(size_t)j * nx + i] != 0.f) x[(size_t)j * nx + i] -= mean;
    }
}

// Plain 16-byte-per-lane copy: the bandwidth reference and the byte-counter
// calibration kernel.
__global__ __launch_bounds__(kBlock) void k_copy16(const float4* __restrict__ src, float4* __restrict__ dst,
                                                   int64_t n16) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k < n16) dst[k] = src[k];
}

void launch_copy16(const void* src, void* dst, int64_t n16, hipStream_t s) {
  const int64_t blocks = (n16 + kBlock - 1) / kBlock;
  k_copy16<<<(unsigned)blocks, kBlock, 0, s>>>((const float4*)src, (float4*)dst, n16);
}

__global__ void k_set_call(CallArgs* c, const float* f, double* x, int max_iter, double delta2) {
  c->f = f;
  c->x = x;
  c->max_iter = max_iter;
  c->delta2 = delta2;
}

// ---------------------------------------------------------------------------
// Host-side launchers (template dispatch on the rows-per-wave tile height).
dim3 stencil_grid(const Coef& c, int R, int nb) {
  const int T = ((c.nx + kWave - 1) / kWave) * ((c.ny + kWaves * R - 1) / (kWaves * R));
  return dim3(8 * ((T + 7) / 8), 1, nb);
}

template <int R>
static dim3 grid_of(const Coef& c, int nb) {
  return stencil_grid(c, R, nb);
}

#define PPE_DISPATCH_R(R, ...)                     \
  switch (R) {                                     \
    case 2: { constexpr int RR = 2; __VA_ARGS__; } break;   \
    case 4: { constexpr int RR = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int RR = 8; __VA_ARGS__; } break;   \
    default: { constexpr int RR = 16; __VA_ARGS__; } break; \
  }

// f = b / (cell area), one thread per cell.
__global__ __launch_bounds__(256) void k_rhs_to_source(Coef c, int64_t n, const float* b, float* f) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= n) return;
  const int64_t cell = q % ((int64_t)c.nx * c.ny);
  const int j = (int)(cell / c.nx), i = (int)(cell - (int64_t)j * c.nx);
  f[q] = (float)((double)b[q] / (c.hx64[i] * c.hy64[j]));
}

void launch_rhs_to_source(const Coef& c, int nb, const float* b, float* f, hipStream_t s) {
  const int64_t n = (int64_t)c.nx * c.ny * nb;
  k_rhs_to_source<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(c, n, b, f);
}

void launch_apply_f32(const Coef& c, int nb, const float* x, float* y, int R, hipStream_t s) {
  if (c.fl) {
    PPE_DISPATCH_R(R, k_apply<float, RR, true><<<grid_of<RR>(c, nb), kBlock, 0, s>>>(c, x, y));
  } else {
    PPE_DISPATCH_R(R, k_apply<float, RR, false><<<grid_of<RR>(c, nb), kBlock, 0, s>>>(c, x, y));
  }
}
void launch_apply_f64(const Coef& c, int nb, const double* x, double* y, int R, hipStream_t s) {
  if (c.fl) {
    PPE_DISPATCH_R(R, k_apply<double, RR, true><<<grid_of<RR>(c, nb), kBlock, 0, s>>>(c, x, y));
  } else {
    PPE_DISPATCH_R(R, k_apply<double, RR, false><<<grid_of<RR>(c, nb), kBlock, 0, s>>>(c, x, y));
  }
}

void launch_set_call(CallArgs* c, const float* f, double* x, int max_iter, double delta2,
                     hipStream_t s) {
  k_set_call<<<1, 1, 0, s>>>(c, f, x, max_iter, delta2);
}

void launch_rhs(const PcgArgs& a, int nb, hipStream_t s) {
  const dim3 g = stencil_grid(a.c, a.R, nb);
  k_rhs_sum<<<g, kBlock, 0, s>>>(a);
  k_rhs_norm<<<g, kBlock, 0, s>>>(a);
}

// Kernel variant (PcKind): 0 none, 1 Jacobi, 2 a supplied z (multigrid);
// 3, 4: none, Jacobi on the solid-mask operator.
static int pc_of(const PcgArgs& a) {
  if (a.mg || a.icq) return 2;
  return (a.c.fl ? 3 : 0) + (a.jacobi ? 1 : 0);
}

#define PPE_DISPATCH_PC(pc, R, ...)                                   \
  switch (pc) {                                                       \
    case 4: { constexpr int PP = 4; PPE_DISPATCH_R(R, __VA_ARGS__); } break; \
    case 3: { constexpr int PP = 3; PPE_DISPATCH_R(R, __VA_ARGS__); } break; \
    case 2: { constexpr int PP = 2; PPE_DISPATCH_R(R, __VA_ARGS__); } break; \
    case 1: { constexpr int PP = 1; PPE_DISPATCH_R(R, __VA_ARGS__); } break; \
    default: { constexpr int PP = 0; PPE_DISPATCH_R(R, __VA_ARGS__); } break; \
  }

// z = M^-1 r for the preconditioners applied by their own kernels after
// every pass that changes r (multigrid V-cycle, red-black IC(0)).
static void launch_pc(const PcgArgs& a, int nb, hipStream_t s) {
  if (a.mg) launch_vcycle(a, nb, s);
  else if (a.icq) launch_ic(a, nb, s);
}

void launch_pcg_setup(const PcgArgs& a, int nb, hipStream_t s) {
  const dim3 g = stencil_grid(a.c, a.R, nb);
  launch_rhs(a, nb, s);
  PPE_DISPATCH_PC(pc_of(a), a.R, k_pcg_init<RR, PP><<<g, kBlock, 0, s>>>(a));
  launch_pc(a, nb, s);
}

// One CG iteration (or reliable-update pass) of the two-phase form; with the
// multigrid preconditioner the V-cycle then turns the new residual into z
// and leaves the partial sums of r.z where phase A reads them.
void launch_pcg_pair(const PcgArgs& a, int nb, int par, int force, int force_restart, hipStream_t s) {
  const dim3 g = stencil_grid(a.c, a.R, nb);
  PPE_DISPATCH_PC(pc_of(a), a.R, k_pcg_a<RR, PP><<<g, kBlock, 0, s>>>(a, par, force, force_restart);
                  k_pcg_b<RR, PP><<<g, kBlock, 0, s>>>(a, par));
  launch_pc(a, nb, s);
}

void launch_pcg_phase_a(const PcgArgs& a, int nb, int par, hipStream_t s) {
  const dim3 g = stencil_grid(a.c, a.R, nb);
  PPE_DISPATCH_PC(pc_of(a), a.R, k_pcg_a<RR, PP><<<g, kBlock, 0, s>>>(a, par, 0, 0));
}

void launch_pcg_phase_b(const PcgArgs& a, int nb, int par, hipStream_t s) {
  const dim3 g = stencil_grid(a.c, a.R, nb);
  PPE_DISPATCH_PC(pc_of(a), a.R, k_pcg_b<RR, PP><<<g, kBlock, 0, s>>>(a, par));
  launch_pc(a, nb, s);
}

// One phase launch whose own dispatch carries the start/stop events, so the
// elapsed time between them is the kernel's execution only (with the
// multigrid preconditioner, the V-cycle follows phase B untimed).
void launch_pcg_phase_timed(const PcgArgs& a, int nb, int par, int phase, hipStream_t s, hipEvent_t e0,
                            hipEvent_t e1) {
  const dim3 g = stencil_grid(a.c, a.R, nb);
  if (phase == 0) {
    PPE_DISPATCH_PC(pc_of(a), a.R,
                    hipExtLaunchKernelGGL(k_pcg_a<RR, PP>, g, dim3(kBlock), 0, s, e0, e1, 0, a, par, 0, 0));
  } else {
    PPE_DISPATCH_PC(pc_of(a), a.R, hipExtLaunchKernelGGL(k_pcg_b<RR, PP>, g, dim3(kBlock), 0, s, e0, e1, 0, a, par));
    launch_pc(a, nb, s);
  }
}

void launch_direction(const PcgArgs& a, int nb, int mode, float* e, hipStream_t s) {
  const dim3 g = stencil_grid(a.c, a.R, nb);
  PPE_DISPATCH_R(a.R, k_direction<RR><<<g, kBlock, 0, s>>>(a, mode, e));
}

void launch_dlsm_step(const PcgArgs& a, int nb, int par, hipStream_t s) {
  const dim3 g = stencil_grid(a.c, a.R, nb);
  PPE_DISPATCH_R(a.R, k_dlsm_a<RR><<<g, kBlock, 0, s>>>(a, par); k_dlsm_b<RR><<<g, kBlock, 0, s>>>(a, par));
  if (a.hist) k_hist_dlsm<<<dim3(1, 1, nb), kBlock, 0, s>>>(a);
}

void launch_mark(const PcgArgs& a, int nb, int cat, hipStream_t s) { k_mark<<<1, 1, 0, s>>>(a, nb, cat); }

void launch_hist_cg(const PcgArgs& a, int nb, int par, hipStream_t s) {
  if (a.hist) k_hist_cg<<<dim3(1, 1, nb), kBlock, 0, s>>>(a, par);
}

__global__ void k_zero_flags(int32_t* flags, int nb) {
  for (int s = threadIdx.x; s < nb; s += blockDim.x) flags[s] = DONE_NO;
}

void launch_zero_flags(int32_t* flags, int nb, hipStream_t s) { k_zero_flags<<<1, 256, 0, s>>>(flags, nb); }

void launch_pcg_finish(const PcgArgs& a, int nb, hipStream_t s) {
  const dim3 g = stencil_grid(a.c, a.R, nb);
  k_x_sum<<<g, kBlock, 0, s>>>(a);
  k_x_shift<<<g, kBlock, 0, s>>>(a);
}

}  // namespace ppe
