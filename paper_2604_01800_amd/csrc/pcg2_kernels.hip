// Two-iteration Jacobi-PCG: one launch and one grid-wide reduction per two CG
// iterations (the s-step form of CG with s = 2; HIP, gfx950).
//
// A launch starts from r_k, p_{k-1} and eleven sums over the grid, reduced
// from the partials of the launch before it. With M = D^-1 and the basis
//   u0 = z_k = M r_k,  u1 = M A u0,  v0 = p_{k-1},  v1 = M A v0,
// the sums are
//   gamma = r.z,  delta = u0.A u0,  zeta = u0.A v0,  pi = v0.A v0,
//   a = u0.A u1,  b = u0.A v1,  c = v0.A v1,
//   d = u1.A u1,  e = u1.A v1,  f = v1.A v1,  and |r|^2
// (every other inner product of the basis that the two steps need equals one
// of these because A and M are symmetric and M D = I). The textbook PCG
// recurrences (Saad, Alg. 9.1) then give, before any vector is touched,
//   beta_{k-1} = gamma / gamma_{k-1},  p_k = u0 + beta v0,
//   alpha_k    = gamma / (delta + 2 beta zeta + beta^2 pi),
//   z_{k+1}    = u0 - alpha u1 - alpha beta v1,
//   gamma_{k+1} = r_{k+1}.z_{k+1}
//              = gamma - 2 alpha (delta + beta zeta)
//                + alpha^2 (a + 2 beta b + beta^2 c),
//   beta_k     = gamma_{k+1} / gamma,
//   p_{k+1}    = (1 + beta_k) u0 - alpha u1 + beta beta_k v0 - alpha beta v1,
//   alpha_{k+1} = gamma_{k+1} / p_{k+1}.A p_{k+1}  (a quadratic form in the sums).
// These are identities of bilinear forms, so the iterates equal the
// one-iteration form's in exact arithmetic. The vectors themselves follow the
// ordinary recurrences
//   s = A p_k,  r_{k+1} = r_k - alpha_k s,  p_{k+1} = M r_{k+1} + beta_k p_k,
//   r_{k+2} = r_{k+1} - alpha_{k+1} A p_{k+1},  x_c += alpha_k p_k + alpha_{k+1} p_{k+1},
// and the launch ends with the eleven partial sums for z_{k+2} and p_{k+1}.
//
// Each wavefront owns 56 columns and R rows and holds a halo of 4 cells on
// every side (64 lanes x R + 8 rows): each of the four stencil levels of a
// launch (A p_k, A p_{k+1}, A z_{k+2}, A u1 and A v1) eats one cell of halo.
// The rows are streamed through the stages in one unrolled pass, so that each
// stage keeps a window of three rows; east and west neighbours are DPP wave
// shifts, and lanes whose values have lost a neighbour are simply not owned.
// HBM traffic per cell and launch: read r, p, x_c and write them (24 B), the
// same as one iteration of the one-iteration form.
//
// Reliable updates use the one-iteration form's three launches: FLUSH adds x_c
// into the FP64 solution, TRUE recomputes r = b - A x in FP64 (the convergence
// judge), and SUMS runs the CG pipeline with zero step lengths and a kept
// direction, which leaves r and p unchanged and forms the eleven sums.
#include <hip/hip_ext.h>

#include "common.hpp"
#include "kernels.hpp"
#include "stencil.hpp"

namespace ppe {

constexpr int kSums2 = 11;
constexpr int kH2 = 4;                  // halo depth of a launch (cells)
constexpr int kOwn2 = kWave - 2 * kH2;  // columns owned by a wavefront
constexpr int kPre = 16;                // partials per thread loaded ahead (P2 <= 256 in one go)

// The CG pipeline's stores write through the L2 (coherence bits sc0 sc1):
// r, p and x_c reach memory while the launch runs, instead of in the L2
// write-back at the kernel boundary that the next launch waits for.
__device__ __forceinline__ void bstore_wt(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)off, 0, 17);
}

// Workgroup sums of N values per thread, stored by one thread per sum into
// part[m][blk] ([N][P]), written through the L2 like the vectors (every
// workgroup of the next launch reads them first). The values go through LDS
// (lds: N * kBlock doubles): thread 16m + c adds threads c, c + 16, ...,
// c + 240 of sum m, and the 16-lane row adds those. Fixed order; needs
// 16 N <= kBlock.
template <int N>
__device__ __forceinline__ void store_sums16(const double (&v)[N], double* lds, double* __restrict__ part, int P,
                                             int blk) {
  static_assert(16 * N <= kBlock, "one 16-lane row per sum");
  typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
  const int t = threadIdx.x;
#pragma unroll
  for (int m = 0; m < N; ++m) lds[m * kBlock + t] = v[m];
  __syncthreads();
  if (t < 16 * N) {
    const int m = t >> 4, c = t & 15;
    const double* l = lds + m * kBlock + c;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kBlock / 16; ++k) s += l[16 * k];
    s = row_sum16(s);
    if (c == 0) {
      const auto pr = make_rsrc(part, (uint64_t)N * P * 8);
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, s), pr, (int)(((uint32_t)m * P + blk) * 8), 0, 17);
    }
  }
}

// Sums of solve s (of nbs solves sharing a.part2) written by launch parity par.
__device__ __forceinline__ double* sums2_of(const PcgArgs& a, int par, int s, int nbs) {
  return a.part2 + ((size_t)par * nbs + s) * kSums2 * a.P2;
}

// Tile placement of this form: tiles of 56 columns x 4R rows, XCD banded as
// for the 64-column tiles. i0 is the column of lane 0, 4 columns west of the
// first owned column.
__device__ __forceinline__ TileXY tile2_xy_at(int nx, int ny, int R, int b) {
  const int gxt = (nx + kOwn2 - 1) / kOwn2;
  const int gyt = (ny + kWaves * R - 1) / (kWaves * R);
  const int T = gxt * gyt;
  const int per = (T + 7) / 8;
  int t = (b & 7) * per + (b >> 3);
  TileXY o;
  o.valid = t < T;
  if (!o.valid) t = 0;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  o.i0 = (t % gxt) * kOwn2 - kH2;
  o.j0 = ((t / gxt) * kWaves + w) * R;
  return o;
}

__device__ __forceinline__ float lane_f32(float v, int q) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), q));
}

// Lane i receives lane i+1 (shl) or lane i-1 (shr) by a DPP wave shift;
// lanes 63 and 0 receive 0.
__device__ __forceinline__ float shl1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ float shr1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}

// Coefficients of one row in one lane: the east and west face weights times
// the row height (cE, and -cW) and the reciprocal diagonal. The weights of
// the faces between rows (times the column width) are kept per face: cF[q]
// for the face below row q, so row q has south weight cF[q] and north weight
// cF[q + 1].
struct RowW {
  float cE, ncW, mi;
};

// (A v) at a cell from its east difference dE = v - v_east (the west
// difference is minus the east difference of the lane to the west) and the
// differences dN = v - v_north of this row and dNs of the row below:
//   A v = cE dE + cW (v - v_west) + cN (v - v_north) + cS (v - v_south).
__device__ __forceinline__ float stencil_d(const RowW& w, float cN, float cS, float dE, float dN, float dNs) {
  float t = w.cE * dE;
  t += w.ncW * shr1(dE);
  t = fmaf(cN, dN, t);
  return fmaf(-cS, dNs, t);
}

template <int R, bool JAC>
__device__ __forceinline__ void pcg2_body(const PcgArgs& a, int s, int nbs, int blk, int par, double* lds,
                                          double* lds_red) {
  constexpr int Q = R + 2 * kH2;  // rows held by a wavefront: j0-4 .. j0+R+3
  const int nx = a.c.nx, ny = a.c.ny;
  SolveState* st = a.st + s;
  const int pm = par ^ 1;
  const size_t off = (size_t)s * a.N;
  const float* __restrict__ rin = (pm ? a.r1 : a.r) + off;
  float* __restrict__ rout = (par ? a.r1 : a.r) + off;
  const float* __restrict__ pin = (pm ? a.p1 : a.p0) + off;
  float* __restrict__ pout = (par ? a.p1 : a.p0) + off;
  float* __restrict__ xc = a.xc + off;
  const int lane = threadIdx.x & (kWave - 1);
  const TileXY tl = tile2_xy_at(nx, ny, R, blk);
  const int i = tl.i0 + lane, j0 = tl.j0;
  const bool inx = tl.valid && i >= 0 && i < nx;
  const bool own = inx && lane >= kH2 && lane < kWave - kH2;

  // Byte offsets of cells: a lane part (kOOB for columns off the grid, or not
  // owned) plus a row part (kOOB for rows off the grid, a scalar), added with
  // unsigned saturation, so any part off the grid gives an out-of-range
  // offset: the buffer access reads 0 or is dropped.
  const uint32_t lane4 = inx ? (uint32_t)i * 4u : kOOB, own4 = own ? (uint32_t)i * 4u : kOOB;
  auto row4 = [&](int j) { return (j >= 0 && j < ny) ? (uint32_t)(j * nx) * 4u : kOOB; };
  auto at = [](uint32_t l, uint32_t r) { return __builtin_elementwise_add_sat(l, r); };

  // Loads first: the previous launch's partial sums (their scalars gate all
  // the arithmetic, and loads complete in issue order), then r and p on all
  // Q rows and x_c on the owned rows.
  double pre[kPre];
  sums16_load<kSums2, kPre>(sums2_of(a, pm, s, nbs), a.P2, pre);
  __builtin_amdgcn_sched_barrier(0);  // keep these loads ahead of the tile loads
  const uint64_t vbytes = (uint64_t)a.N * 4;
  const auto rsr = make_rsrc(rin, vbytes), psr = make_rsrc(pin, vbytes), xsr = make_rsrc(xc, vbytes);
  float ro[Q], po[Q], xcv[R];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const uint32_t o = at(lane4, row4(j0 - kH2 + q));
    ro[q] = bload(rsr, o);
    po[q] = bload(psr, o);
  }
#pragma unroll
  for (int q = 0; q < R; ++q) xcv[q] = bload(xsr, at(own4, row4(j0 + q)));
  // Row coefficients of rows j0-4 .. j0+R+3 (faces j0-4 .. j0+R+4): lane q
  // holds those of row j0-4+q (the padded arrays read 0 off the grid), and
  // each row's values are taken with readlane where the row is processed, so
  // the R+8 rows do not occupy scalar registers all at once.
  const int lq = lane < Q ? lane : Q;
  const float hyv = a.c.hy[j0 - kH2 + lq], gyv = a.c.gy[j0 - kH2 + lq];
  const float hx = a.c.hx[i], gw = a.c.gx[i], ge = a.c.gx[i + 1];
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
  double sum[kSums2];
  sums16_finish<kSums2, kPre>(sums2_of(a, pm, s, nbs), a.P2, pre, lds_red, sum);
  if (__builtin_expect(dprev != 0, 0)) {
    if (leader) st->dflag[par] = dprev;
    return;
  }

  // What this launch does, and the step scalars of the CG pipeline:
  //   p_k = c0 z_k + beta p_{k-1},  r_{k+1} = r_k - alpha A p_k,
  //   p_{k+1} = cz z_{k+1} + beta1 p_k,  r_{k+2} = r_{k+1} - alpha1 A p_{k+1}.
  int todo = MODE_CG, rst_next = 0;
  double c0 = 1.0, beta = 0.0, alpha = 0.0, cz = 1.0, beta1 = 1.0, alpha1 = 0.0;
  if (__builtin_expect(pmode == MODE_FLUSH, 0)) {
    todo = MODE_TRUE;
  } else if (__builtin_expect(pmode == MODE_TRUE, 0)) {
    const double rr = sum[10];
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
    // SUMS: r and p kept, x_c unchanged.
    todo = MODE_SUMS;
    rr_ru = rr;
    c0 = 0.0;
    beta = 1.0;
    cz = 0.0;
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
    const double gam = sum[0], del = sum[1], zet = sum[2], pip = sum[3];
    const double sa = sum[4], sb = sum[5], sc = sum[6], sd = sum[7], se = sum[8], sf = sum[9], rr = sum[10];
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
    int nit = 2;
    double gam_next = gam;
    if (!flush) {
      bool two = it + 2 <= max_iter;
      if (two) {
        const double g1 = gam - 2.0 * alpha * (del + beta * zet) + alpha * alpha * (sa + 2.0 * beta * sb + beta * beta * sc);
        const double b1 = g1 / gam;
        const double k0 = 1.0 + b1, k1 = -alpha, k2 = beta * b1, k3 = -alpha * beta;
        const double pap1 = k0 * k0 * del + k1 * k1 * sd + k2 * k2 * pip + k3 * k3 * sf +
                            2.0 * (k0 * k1 * sa + k0 * k2 * zet + k0 * k3 * sb + k1 * k2 * sb + k1 * k3 * se +
                                   k2 * k3 * sc);
        const double a1 = g1 / pap1;
        two = g1 > 0.0 && pap1 > 0.0 && isfinite(a1) && isfinite(b1);
        if (two) {
          beta1 = b1;
          alpha1 = a1;
          gam_next = g1;
        }
      }
      if (!two) {  // one iteration: p_{k+1} = p_k and r_{k+2} = r_{k+1}
        nit = 1;
        cz = 0.0;
        beta1 = 1.0;
        alpha1 = 0.0;
      }
    }
    if (flush) todo = MODE_FLUSH;
    if (leader && todo == MODE_CG) {
      st->mode[par] = MODE_CG;
      st->it[par] = it + nit;
      st->it_cg[par] = itcg + nit;
      st->n_ru[par] = nru;
      st->rho[par] = gam_next;
      st->rr_ru[par] = rr_ru;
      st->rr_last[par] = rr;
      st->restart[par] = 0;
      st->alpha[par] = alpha1;
      st->dflag[par] = DONE_NO;
    }
  }

  if (__builtin_expect(todo == MODE_FLUSH, 0)) {
    // Reliable update, part 1: x += x_c in FP64, x_c = 0, p carried over.
    const auto x64 = make_rsrc(uniform_ptr(a.call->x) + off, (uint64_t)a.N * 8);
    const auto pso = make_rsrc(pout, vbytes);
    double xv[R];
#pragma unroll
    for (int q = 0; q < R; ++q) xv[q] = bload64(x64, cell_off8(own, j0 + q, ny, nx, i));
#pragma unroll
    for (int q = 0; q < R; ++q) {
      bstore64(x64, cell_off8(own, j0 + q, ny, nx, i), xv[q] + (double)xcv[q]);
      const uint32_t o = cell_off(own, j0 + q, ny, nx, i);
      bstore(xsr, o, 0.f);
      bstore(pso, o, po[q + kH2]);
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

  double acc[kSums2];
#pragma unroll
  for (int m = 0; m < kSums2; ++m) acc[m] = 0.0;
  if (__builtin_expect(todo == MODE_TRUE, 0)) {
    // Reliable update, part 2: r = b - A x in FP64 on the owned cells (the x
    // window walks down the column; east and west come from lane shuffles)
    // and |r|^2 in FP64, the convergence judge. p is carried over.
    const auto x64 = make_rsrc(uniform_ptr(a.call->x) + off, (uint64_t)a.N * 8);
    const auto fsr = make_rsrc(uniform_ptr(a.call->f) + off, vbytes);
    const auto rso = make_rsrc(rout, vbytes), pso = make_rsrc(pout, vbytes);
    const double bmean = st->bmean;
    double x_p = bload64(x64, cell_off8(inx, j0 - 1, ny, nx, i));
    double x_c = bload64(x64, cell_off8(inx, j0, ny, nx, i));
#pragma unroll 1
    for (int q = 0; q < R; ++q) {
      const int j = j0 + q;
      const double x_n = bload64(x64, cell_off8(inx, j + 1, ny, nx, i));
      const uint32_t o = cell_off(own, j, ny, nx, i);
      const float fv = bload(fsr, o);
      const double xe = __shfl_down(x_c, 1, kWave), xw = __shfl_up(x_c, 1, kWave);
      const double rv = true_res(a.c, i, j, x_c, xe, xw, x_n, x_p, fv, bmean);
      bstore(rso, o, (float)rv);
      bstore(pso, o, bload(psr, cell_off(own, j, ny, nx, i)));
      acc[10] += (own && j < ny) ? rv * rv : 0.0;
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
  } else {
    // The CG pipeline (CG and SUMS launches), streamed down the rows: at step
    // t, stage 0 forms p_k on row t, stage 1 A p_k, r_{k+1} and p_{k+1} on row
    // t-1, stage 2 A p_{k+1}, r_{k+2}, z_{k+2} and v1 on row t-2 (owned rows
    // are stored here), stage 3 A z_{k+2} and u1 on row t-3, stage 4 A u1 and
    // A v1 on row t-4. Off the grid every value and coefficient is 0 (the
    // reciprocal diagonal is large but finite), so no product leaks in.
    const float fc0 = (float)c0, fbet = (float)beta, falf = (float)alpha;
    const float fcz = (float)cz, fbet1 = (float)beta1, falf1 = (float)alpha1;
    const bool rst = beta == 0.0;
    const auto rso = make_rsrc(rout, vbytes), pso = make_rsrc(pout, vbytes);
    // Per row: coefficients; per field and row: the value and its north
    // difference (value minus the value of the row above).
    RowW W[Q];
    float cF[Q + 1];
    float pk[Q], dpk[Q], r1[Q], pk1[Q], dpk1[Q], z2[Q], dz2[Q], v1[Q], dv1[Q], u1[Q], du1[Q];
    const float gew = ge + gw;
    cF[0] = hx * lane_f32(gyv, 0);
#pragma unroll
    for (int t = 0; t < Q; ++t) {
      {  // coefficients and stage 0 (p_k) on row t
        const float hyq = lane_f32(hyv, t);
        cF[t + 1] = hx * lane_f32(gyv, t + 1);
        W[t].cE = hyq * ge;
        W[t].ncW = -(hyq * gw);
        W[t].mi = JAC ? __builtin_amdgcn_rcpf(fmaxf(fmaf(hyq, gew, cF[t] + cF[t + 1]), 1e-30f)) : 1.f;
        const float z = ro[t] * W[t].mi;
        pk[t] = rst ? fc0 * z : fc0 * z + fbet * po[t];
        if (t >= 1) dpk[t - 1] = pk[t - 1] - pk[t];
      }
      if (t >= 2) {  // stage 1, row q = t - 1: A p_k, r_{k+1}, p_{k+1}
        const int q = t - 1;
        const float s0 = stencil_d(W[q], cF[q + 1], cF[q], pk[q] - shl1(pk[q]), dpk[q], dpk[q - 1]);
        r1[q] = ro[q] - falf * s0;
        pk1[q] = fcz * (r1[q] * W[q].mi) + fbet1 * pk[q];
        if (q >= 2) dpk1[q - 1] = pk1[q - 1] - pk1[q];
      }
      if (t >= 4) {  // stage 2, row q = t - 2: A p_{k+1}, r_{k+2}, z_{k+2}, v1; stores
        const int q = t - 2;
        const float s1 = stencil_d(W[q], cF[q + 1], cF[q], pk1[q] - shl1(pk1[q]), dpk1[q], dpk1[q - 1]);
        const float r2 = r1[q] - falf1 * s1;
        z2[q] = r2 * W[q].mi;
        v1[q] = W[q].mi * s1;
        if (q >= 3) {
          dz2[q - 1] = z2[q - 1] - z2[q];
          dv1[q - 1] = v1[q - 1] - v1[q];
        }
        if (q >= kH2 && q < kH2 + R) {
          const uint32_t o = at(own4, row4(j0 - kH2 + q));
          bstore_wt(rso, o, r2);
          bstore_wt(pso, o, pk1[q]);
          bstore_wt(xsr, o, xcv[q - kH2] + falf * pk[q] + falf1 * pk1[q]);
          const double dr = r2, dz = z2[q], ds = s1, dp = pk1[q], dv = v1[q];
          acc[0] += own ? dr * dz : 0.0;
          acc[2] += own ? dz * ds : 0.0;
          acc[3] += own ? dp * ds : 0.0;
          acc[6] += own ? ds * dv : 0.0;
          acc[10] += own ? dr * dr : 0.0;
        }
      }
      if (t >= 6) {  // stage 3, row q = t - 3: A z_{k+2}, u1
        const int q = t - 3;
        const float az = stencil_d(W[q], cF[q + 1], cF[q], z2[q] - shl1(z2[q]), dz2[q], dz2[q - 1]);
        u1[q] = W[q].mi * az;
        if (q >= 4) du1[q - 1] = u1[q - 1] - u1[q];
        if (q >= kH2 && q < kH2 + R) {
          const double da = az, dz = z2[q], du = u1[q], dv = v1[q];
          acc[1] += own ? dz * da : 0.0;
          acc[4] += own ? da * du : 0.0;
          acc[5] += own ? da * dv : 0.0;
        }
      }
      if (t >= 8) {  // stage 4, row q = t - 4 (an owned row): A u1, A v1
        const int q = t - 4;
        const float au = stencil_d(W[q], cF[q + 1], cF[q], u1[q] - shl1(u1[q]), du1[q], du1[q - 1]);
        const float av = stencil_d(W[q], cF[q + 1], cF[q], v1[q] - shl1(v1[q]), dv1[q], dv1[q - 1]);
        const double du = u1[q], dv = v1[q], dau = au, dav = av;
        acc[7] += own ? du * dau : 0.0;
        acc[8] += own ? dau * dv : 0.0;
        acc[9] += own ? dv * dav : 0.0;
      }
    }
  }
  store_sums16<kSums2>(acc, lds, sums2_of(a, par, s, nbs), a.P2, blk);
}

template <int R, bool JAC>
__global__ __launch_bounds__(kBlock) void k_pcg2(PcgArgs a, int par) {
  __shared__ double lds[kSums2 * kBlock];
  __shared__ double lds_red[kSums2];
  pcg2_body<R, JAC>(a, blockIdx.z, gridDim.z, blockIdx.x, par, lds, lds_red);
}

// Tile heights of this form: those of the other forms plus 20 and 24 rows,
// which let a 1024-row grid fill the CUs with one workgroup each.
// Solves on grids of different sizes in one launch: work[b] = (solve << 20) |
// (workgroup within the solve) for the launch's workgroup b; descs[solve] is
// that solve's argument block (one solve each).
template <int R, bool JAC>
__global__ __launch_bounds__(kBlock) void k_pcg2_multi(const PcgArgs* __restrict__ descs,
                                                       const uint32_t* __restrict__ work, int par) {
  __shared__ double lds[kSums2 * kBlock];
  __shared__ double lds_red[kSums2];
  const uint32_t wv = __builtin_amdgcn_readfirstlane(work[blockIdx.x]);
  pcg2_body<R, JAC>(descs[wv >> 20], 0, 1, (int)(wv & 0xFFFFFu), par, lds, lds_red);
}

#define PPE2_CASES(RV, JV, ...)                                                         \
  switch (RV) {                                                                     \
    case 2: { constexpr int RR = 2; constexpr bool JJ = JV; __VA_ARGS__; } break;   \
    case 4: { constexpr int RR = 4; constexpr bool JJ = JV; __VA_ARGS__; } break;   \
    case 8: { constexpr int RR = 8; constexpr bool JJ = JV; __VA_ARGS__; } break;   \
    case 16: { constexpr int RR = 16; constexpr bool JJ = JV; __VA_ARGS__; } break; \
    case 20: { constexpr int RR = 20; constexpr bool JJ = JV; __VA_ARGS__; } break; \
    default: { constexpr int RR = 24; constexpr bool JJ = JV; __VA_ARGS__; } break; \
  }
#define PPE2_DISPATCH(R, JAC, ...) \
  do {                             \
    if (JAC) {                     \
      PPE2_CASES(R, true, __VA_ARGS__) \
    } else {                       \
      PPE2_CASES(R, false, __VA_ARGS__) \
    }                              \
  } while (0)

dim3 stencil_grid2(const Coef& c, int R, int nb) {
  const int T = ((c.nx + kOwn2 - 1) / kOwn2) * ((c.ny + kWaves * R - 1) / (kWaves * R));
  return dim3(8 * ((T + 7) / 8), 1, nb);
}

// Set-up: right-hand side, then the one-iteration form's initial state (x_c
// and both p buffers zero, state as after a FLUSH of parity 0), so that the
// first launch (parity 1) computes the true residual of the initial guess.
void launch_pcg2_setup(const PcgArgs& a, int nb, hipStream_t s) {
  launch_rhs(a, nb, s);
  launch_pcg1_init(a, nb, s);
  launch_pcg2_step(a, nb, 1, s);
}

void launch_pcg2_step(const PcgArgs& a, int nb, int par, hipStream_t s) {
  const dim3 g = stencil_grid2(a.c, a.R, nb);
  PPE2_DISPATCH(a.R, a.jacobi, k_pcg2<RR, JJ><<<g, kBlock, 0, s>>>(a, par));
}

void launch_pcg2_multi_step(const PcgArgs* descs, const uint32_t* work, int nblocks, int R, bool jacobi, int par,
                            hipStream_t s) {
  PPE2_DISPATCH(R, jacobi, k_pcg2_multi<RR, JJ><<<nblocks, kBlock, 0, s>>>(descs, work, par));
}

void launch_pcg2_step_timed(const PcgArgs& a, int nb, int par, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const dim3 g = stencil_grid2(a.c, a.R, nb);
  PPE2_DISPATCH(a.R, a.jacobi, hipExtLaunchKernelGGL(k_pcg2<RR, JJ>, g, dim3(kBlock), 0, s, e0, e1, 0, a, par));
}

}  // namespace ppe
