/*
 * TEST INFRASTRUCTURE — the FP64 CPU oracle for the pressure Poisson solve.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this library. It shares no code with the GPU library.
 * It is plain, single-threaded FP64 C, written for checking by eye, not speed.
 *
 * The operator (Eq. 7 / Eq. 10, the pressure Poisson matrix M) is read as the
 * cell-centred finite-volume form of -div(grad p) on a tensor-product grid:
 * each interior face contributes weight  w = (face length) / (distance between
 * the two cell centres)  to the two cells it joins, and boundary faces are
 * dropped (homogeneous Neumann). The time step is absorbed into the source.
 *     (A x)_c = sum over interior faces f of c:  w_f (x_c - x_nb(f))
 * The matrix is symmetric positive semi-definite with the constant vector as
 * its null space. The source of -lap p = f becomes b = (cell area) * f, and b
 * is projected onto range(A) by removing its plain mean.
 *
 * Solid-mask mode (mask_mode 1, an option beside the paper's form, in which
 * the obstacle does not enter the matrix): only faces between two fluid cells
 * (mask 0) carry weight, and a solid cell's row is the identity, (A x)_c = x_c.
 * The null space is then the fluid indicator (for a connected fluid region);
 * b = (cell area) f minus its mean over the fluid cells, on fluid cells, and
 * 0 on solid cells.
 *
 * Jacobi-PCG follows the textbook preconditioned CG (Saad, Iterative Methods
 * for Sparse Linear Systems, Alg. 9.1) with D = diag(A). The hybrid solve
 * follows Sec. 2.2: consecutive blocks of at most Num_CG-type CG iterations and
 * Num_DLSM line-search steps along a supplied error direction e
 * (alpha = r.e / e.Me, Eqs. 12-13), checking the residual L2 norm after every
 * iteration. The CG block restarts from the current residual after each
 * line-search block.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t nx, ny;
  const double *xc, *yc, *hx, *hy;
  const uint8_t* mask;  /* [ny][nx], 1 = solid; used in mask_mode 1 only */
  int32_t mask_mode;    /* 0: the mask does not enter A; 1: solid cells are cut out */
} orc_grid;

/* 1 when cell (i, j) takes part in the operator as a fluid cell. */
static int fluid(const orc_grid* g, int i, int j) {
  return g->mask_mode != 1 || g->mask[(size_t)j * g->nx + i] == 0;
}

/* Weight of the face between cells (i,j) and (i+1,j): face length hy[j] over
 * centre distance xc[i+1]-xc[i]. */
static double wface_x(const orc_grid* g, int i, int j) {
  return g->hy[j] / (g->xc[i + 1] - g->xc[i]);
}
/* Weight of the face between cells (i,j) and (i,j+1). */
static double wface_y(const orc_grid* g, int i, int j) {
  return g->hx[i] / (g->yc[j + 1] - g->yc[j]);
}

/* y = A x (x, y: [ny][nx], index j*nx + i). */
void orc_apply(const orc_grid* g, const double* x, double* y) {
  const int nx = g->nx, ny = g->ny;
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      const double xcen = x[(size_t)j * nx + i];
      if (!fluid(g, i, j)) {
        y[(size_t)j * nx + i] = xcen;
        continue;
      }
      double s = 0.0;
      if (i > 0 && fluid(g, i - 1, j)) s += wface_x(g, i - 1, j) * (xcen - x[(size_t)j * nx + i - 1]);
      if (i < nx - 1 && fluid(g, i + 1, j)) s += wface_x(g, i, j) * (xcen - x[(size_t)j * nx + i + 1]);
      if (j > 0 && fluid(g, i, j - 1)) s += wface_y(g, i, j - 1) * (xcen - x[(size_t)(j - 1) * nx + i]);
      if (j < ny - 1 && fluid(g, i, j + 1)) s += wface_y(g, i, j) * (xcen - x[(size_t)(j + 1) * nx + i]);
      y[(size_t)j * nx + i] = s;
    }
  }
}

/* d = diag(A). */
void orc_diag(const orc_grid* g, double* d) {
  const int nx = g->nx, ny = g->ny;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      if (!fluid(g, i, j)) {
        d[(size_t)j * nx + i] = 1.0;
        continue;
      }
      double s = 0.0;
      if (i > 0 && fluid(g, i - 1, j)) s += wface_x(g, i - 1, j);
      if (i < nx - 1 && fluid(g, i + 1, j)) s += wface_x(g, i, j);
      if (j > 0 && fluid(g, i, j - 1)) s += wface_y(g, i, j - 1);
      if (j < ny - 1 && fluid(g, i, j + 1)) s += wface_y(g, i, j);
      d[(size_t)j * nx + i] = s;
    }
}

double orc_dot(int64_t n, const double* a, const double* b) {
  double s = 0.0;
  for (int64_t k = 0; k < n; ++k) s += a[k] * b[k];
  return s;
}

/* b = (cell area) f, then b -= mean(b) (solid-mask mode: over and on the
 * fluid cells only, b = 0 on solid cells). Returns the removed mean. */
double orc_rhs(const orc_grid* g, const float* f, double* b) {
  const int nx = g->nx, ny = g->ny;
  double sum = 0.0;
  int64_t count = 0;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const double v = g->hx[i] * g->hy[j] * (double)f[(size_t)j * nx + i];
      b[(size_t)j * nx + i] = v;
      if (fluid(g, i, j)) {
        sum += v;
        ++count;
      }
    }
  const double mean = sum / (double)count;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      double* bv = &b[(size_t)j * nx + i];
      *bv = fluid(g, i, j) ? *bv - mean : 0.0;
    }
  return mean;
}

typedef struct {
  int32_t converged, iters_total, iters_cg, iters_dlsm, dlsm_rejected, breakdowns;
  double res_final; /* recursive residual L2 norm at exit */
} orc_stats;

/* Error provider: fills e from r (both length n). Returns nonzero on failure. */
typedef int (*orc_provider)(void* ctx, const double* r, double* e);

static void record(double* hist, int32_t cap, int32_t k, double v) {
  if (hist && k < cap) hist[k] = v;
}

/* z = M^-1 r for the preconditioner in use: diagonal (dinv) or a supplied
 * operator (pc). Returns nonzero when the supplied operator fails. */
static int precond_apply(int64_t n, const double* dinv, orc_provider pc, void* pc_ctx, const double* r,
                         double* z) {
  if (pc) return pc(pc_ctx, r, z);
  for (int64_t m = 0; m < n; ++m) z[m] = dinv[m] * r[m];
  return 0;
}

/*
 * Hybrid solve (Sec. 2.2). num_dlsm = 0 (or provider = NULL) gives plain PCG
 * with no restarts. precond: 0 = none (vanilla CG), 1 = Jacobi, 2 = the
 * supplied symmetric positive (semi-)definite operator pc (z = pc(r), e.g. a
 * multigrid V-cycle).
 * tol_kind: 0 = stop when ||r|| <= tol ||b||, 1 = stop when ||r|| <= tol.
 * tol <= 0 runs exactly max_iter iterations. x holds x0 on entry.
 * hist[0] = initial residual norm, hist[k] = norm after iteration k.
 * Returns 0 when converged, 1 otherwise.
 */
int orc_hybrid_pc(const orc_grid* g, const double* b, double* x, int precond,
                  double tol, int tol_kind, int max_iter, int num_cg, int num_dlsm,
                  orc_provider prov, void* ctx, orc_provider pc, void* pc_ctx,
                  orc_stats* st, double* hist, int32_t hist_cap) {
  const int64_t n = (int64_t)g->nx * g->ny;
  double* r = (double*)malloc(sizeof(double) * n);
  double* z = (double*)malloc(sizeof(double) * n);
  double* p = (double*)malloc(sizeof(double) * n);
  double* q = (double*)malloc(sizeof(double) * n);
  double* dinv = (double*)malloc(sizeof(double) * n);
  double* e = (double*)malloc(sizeof(double) * n);
  orc_stats s;
  memset(&s, 0, sizeof(s));

  orc_diag(g, dinv);
  for (int64_t k = 0; k < n; ++k) dinv[k] = precond == 1 ? 1.0 / dinv[k] : 1.0;
  if (precond != 2) pc = NULL;
  int pc_failed = 0;

  orc_apply(g, x, q);
  for (int64_t k = 0; k < n; ++k) r[k] = b[k] - q[k];
  const double bnorm = sqrt(orc_dot(n, b, b));
  const double thr = tol <= 0.0 ? -1.0 : (tol_kind == 1 ? tol : tol * bnorm);
  double rnorm = sqrt(orc_dot(n, r, r));
  record(hist, hist_cap, 0, rnorm);
  int k = 0;
  int hybrid = (prov != NULL && num_dlsm > 0);
  if (!hybrid) num_cg = max_iter;
  int done = rnorm <= thr;

  while (!done && k < max_iter) {
    /* CG block, restarted from the current residual. */
    if (precond_apply(n, dinv, pc, pc_ctx, r, z)) { pc_failed = 1; break; }
    memcpy(p, z, sizeof(double) * n);
    double rho = orc_dot(n, r, z);
    for (int c = 0; c < num_cg && !done && k < max_iter; ++c) {
      orc_apply(g, p, q);
      const double pq = orc_dot(n, p, q);
      if (!(pq > 0.0)) { /* breakdown: p is in the null space or r = 0 */
        s.breakdowns++;
        break;
      }
      const double alpha = rho / pq;
      for (int64_t m = 0; m < n; ++m) {
        x[m] += alpha * p[m];
        r[m] -= alpha * q[m];
      }
      ++k;
      s.iters_cg++;
      rnorm = sqrt(orc_dot(n, r, r));
      record(hist, hist_cap, k, rnorm);
      if (rnorm <= thr) { done = 1; break; }
      if (precond_apply(n, dinv, pc, pc_ctx, r, z)) { pc_failed = 1; break; }
      const double rho_new = orc_dot(n, r, z);
      const double beta = rho_new / rho;
      rho = rho_new;
      for (int64_t m = 0; m < n; ++m) p[m] = z[m] + beta * p[m];
    }
    if (!hybrid || pc_failed) break;
    /* Line-search block along the supplied error directions (Eqs. 12-13). */
    for (int d = 0; d < num_dlsm && !done && k < max_iter; ++d) {
      int bad = prov(ctx, r, e) != 0;
      double num = 0.0, den = 0.0, ee = 0.0;
      if (!bad) {
        orc_apply(g, e, q);
        num = orc_dot(n, r, e);
        den = orc_dot(n, e, q);
        ee = orc_dot(n, e, e);
        bad = !isfinite(num) || !isfinite(den) || !(den > 1e-30 * ee);
      }
      ++k;
      if (bad) {
        s.dlsm_rejected++;
        record(hist, hist_cap, k, rnorm);
        continue;
      }
      const double alpha = num / den;
      for (int64_t m = 0; m < n; ++m) {
        x[m] += alpha * e[m];
        r[m] -= alpha * q[m];
      }
      s.iters_dlsm++;
      rnorm = sqrt(orc_dot(n, r, r));
      record(hist, hist_cap, k, rnorm);
      if (rnorm <= thr) done = 1;
    }
  }
  s.iters_total = k;
  s.converged = done;
  s.res_final = rnorm;
  if (st) *st = s;
  free(r); free(z); free(p); free(q); free(dinv); free(e);
  return done ? 0 : 1;
}

int orc_hybrid(const orc_grid* g, const double* b, double* x, int precond,
               double tol, int tol_kind, int max_iter, int num_cg, int num_dlsm,
               orc_provider prov, void* ctx, orc_stats* st, double* hist,
               int32_t hist_cap) {
  return orc_hybrid_pc(g, b, x, precond, tol, tol_kind, max_iter, num_cg, num_dlsm, prov, ctx, NULL, NULL,
                       st, hist, hist_cap);
}

/* Plain PCG: the hybrid with no line-search block. */
int orc_pcg(const orc_grid* g, const double* b, double* x, int precond,
            double tol, int tol_kind, int max_iter, orc_stats* st, double* hist,
            int32_t hist_cap) {
  return orc_hybrid(g, b, x, precond, tol, tol_kind, max_iter, max_iter, 0,
                    NULL, NULL, st, hist, hist_cap);
}

/* Subtract the plain mean (the component along the null space). */
void orc_remove_mean(int64_t n, double* x) {
  double s = 0.0;
  for (int64_t k = 0; k < n; ++k) s += x[k];
  s /= (double)n;
  for (int64_t k = 0; k < n; ++k) x[k] -= s;
}
