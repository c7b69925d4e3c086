// Host side of the multigrid preconditioner: the level hierarchy of a
// problem (coarse 1D coefficient arrays, level buffers) and the factored
// separable solve of the coarsest level, built once per (levels, batch size)
// and reused by every solve, as the paper reuses its preconditioner across
// time steps (Sec. 2.5).
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <vector>

#include "mg_internal.hpp"

extern "C" ppe_status ppe_tridiag_eigh(int32_t n, const double* alpha, const double* beta, double* theta, double* U);

namespace ppe {

void mg_free(MgData* m) {
  if (!m) return;
  for (void* q : m->owned) dev_free(q);
  delete m;
}

namespace {

// Tile height of a coarse level's stencil kernels by its size.
int level_rows(int64_t cells) {
  if (cells >= ((int64_t)1 << 20)) return 8;
  if (cells >= ((int64_t)1 << 17)) return 4;
  return 2;
}

template <typename T>
T* alloc_n(MgData* m, size_t n) {
  T* q = (T*)dev_alloc(sizeof(T) * (n ? n : 1));
  if (q) m->owned.push_back(q);
  return q;
}

// Galerkin coarsening of one axis (piecewise-constant aggregation of pairs):
// merged widths, and the fine face factor at every surviving face.
void coarsen_axis(const std::vector<double>& h, const std::vector<double>& g, std::vector<double>& hc,
                  std::vector<double>& gc) {
  const int n = (int)h.size() / 2;
  hc.resize(n);
  gc.resize(n + 1);
  for (int i = 0; i < n; ++i) hc[i] = h[2 * i] + h[2 * i + 1];
  for (int k = 0; k <= n; ++k) gc[k] = g[2 * k];
}

}  // namespace

ppe_status mg_ensure(ppe_problem* p, int L, int nb, int R0, hipStream_t s) {
  MgData* m = p->mg;
  // the fine level's tiling only matters when it writes the coarsest sums
  if (m && m->L == L && m->nb >= nb && (L != 2 || m->R0 == R0)) return PPE_OK;
  mg_free(m);
  p->mg = nullptr;
  const int cnx = p->nx >> (L - 1), cny = p->ny >> (L - 1);
  if (cnx > kMgCoarseMaxNx || cny > kMgCoarseMaxNy)
    return set_error(PPE_ERR_UNSUPPORTED,
                     "the coarsest multigrid level (%d x %d) exceeds %d x %d cells: use more levels", cnx, cny,
                     kMgCoarseMaxNx, kMgCoarseMaxNy);
  static std::atomic<uint64_t> next_uid{1};
  m = new MgData();
  m->uid = next_uid.fetch_add(1);
  m->L = L;
  m->nb = nb;
  m->R0 = R0;
  m->lv.resize(L);
  auto fail = [&](const char* what) {
    mg_free(m);
    return set_error(PPE_ERR_HIP, "multigrid set-up: %s", what);
  };
  // level arrays in FP64 on the host
  std::vector<double> hx(p->hx), hy(p->hy), gx(p->nx + 1, 0.0), gy(p->ny + 1, 0.0), xc(p->xc), yc(p->yc);
  for (int k = 1; k < p->nx; ++k) gx[k] = 1.0 / (p->xc[k] - p->xc[k - 1]);
  for (int k = 1; k < p->ny; ++k) gy[k] = 1.0 / (p->yc[k] - p->yc[k - 1]);
  std::vector<std::vector<double>> h64s(L);
  std::vector<std::vector<float>> h32s(L);
  for (int l = 0; l < L; ++l) {
    MgLevel& v = m->lv[l];
    v.nx = (int)hx.size();
    v.ny = (int)hy.size();
    const int64_t N = (int64_t)v.nx * v.ny;
    if (l == 0) {
      v.c = p->coef;
      v.R = R0;
    } else {
      // centres of merged cells (used by nothing in the V-cycle; kept consistent)
      std::vector<double> xcc(v.nx), ycc(v.ny);
      for (int i = 0; i < v.nx; ++i) xcc[i] = 0.5 * (xc[2 * i] + xc[2 * i + 1]);
      for (int j = 0; j < v.ny; ++j) ycc[j] = 0.5 * (yc[2 * j] + yc[2 * j + 1]);
      xc.swap(xcc);
      yc.swap(ycc);
      ppe_status st = coef_upload(v.nx, v.ny, hx.data(), hy.data(), gx.data(), gy.data(), xc.data(), yc.data(), s,
                                  h64s[l], h32s[l], &v.dev_coef, &v.c);
      if (v.dev_coef) m->owned.push_back(v.dev_coef);
      if (st != PPE_OK) {
        mg_free(m);
        return st;
      }
      v.R = level_rows(N * nb);
      v.b = alloc_n<float>(m, (size_t)N * nb);
      v.x = alloc_n<float>(m, (size_t)N * nb);
      v.y = alloc_n<float>(m, (size_t)N * nb);
      v.d = alloc_n<float>(m, (size_t)N * nb);
      if (!v.b || !v.x || !v.y || !v.d) return fail("level buffers");
    }
    v.P = (int)stencil_grid(v.c, v.R, 1).x;
    if (l + 1 < L) {
      std::vector<double> hc, gc;
      coarsen_axis(hx, gx, hc, gc);
      hx.swap(hc);
      gx.swap(gc);
      coarsen_axis(hy, gy, hc, gc);
      hy.swap(hc);
      gy.swap(gc);
    }
  }
  const int64_t N0 = (int64_t)p->nx * p->ny;
  m->z = alloc_n<float>(m, (size_t)N0 * nb);
  m->d0 = alloc_n<float>(m, (size_t)N0 * nb);
  m->y0 = alloc_n<float>(m, (size_t)N0 * nb);
  if (!m->z || !m->d0 || !m->y0) return fail("fine-level buffers");

  // Coarsest level: hx, gx, hy, gy now hold its arrays.
  const int nxc = (int)hx.size(), nyc = (int)hy.size();
  m->nxc = nxc;
  m->nyc = nyc;
  // Generalised eigenvectors of one axis, T v = lam H v with v^T H v = 1,
  // through the symmetric S = H^-1/2 T H^-1/2 (tridiagonal); ascending, so
  // mode 0 is the constant (lam = 0).
  auto axis_eig = [&](const std::vector<double>& h, const std::vector<double>& g, std::vector<double>& lam,
                      std::vector<double>& V) -> ppe_status {
    const int n = (int)h.size();
    std::vector<double> sd(n), so(n > 1 ? n - 1 : 0), U((size_t)n * n);
    lam.resize(n);
    for (int i = 0; i < n; ++i) sd[i] = (g[i] + g[i + 1]) / h[i];
    for (int i = 0; i + 1 < n; ++i) so[i] = -g[i + 1] / std::sqrt(h[i] * h[i + 1]);
    ppe_status st = ppe_tridiag_eigh(n, sd.data(), so.data(), lam.data(), U.data());
    if (st != PPE_OK) return st;
    V.resize((size_t)n * n);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) V[(size_t)i * n + k] = U[(size_t)i * n + k] / std::sqrt(h[i]);
    lam[0] = 0.0;  // the constant mode
    return PPE_OK;
  };
  std::vector<double> lam, mu, phi, psi;
  ppe_status est = axis_eig(hx, gx, lam, phi);
  if (est == PPE_OK) est = axis_eig(hy, gy, mu, psi);
  if (est != PPE_OK) {
    mg_free(m);
    return est;
  }
  std::vector<double> phiT((size_t)nxc * nxc), psiT((size_t)nyc * nyc), dinv((size_t)nyc * nxc);
  for (int i = 0; i < nxc; ++i)
    for (int k = 0; k < nxc; ++k) phiT[(size_t)k * nxc + i] = phi[(size_t)i * nxc + k];
  for (int j = 0; j < nyc; ++j)
    for (int k = 0; k < nyc; ++k) psiT[(size_t)k * nyc + j] = psi[(size_t)j * nyc + k];
  for (int j = 0; j < nyc; ++j)
    for (int k = 0; k < nxc; ++k) dinv[(size_t)j * nxc + k] = (j == 0 && k == 0) ? 0.0 : 1.0 / (lam[k] + mu[j]);
  m->phi = alloc_n<double>(m, phi.size());
  m->phiT = alloc_n<double>(m, phiT.size());
  m->psi = alloc_n<double>(m, psi.size());
  m->psiT = alloc_n<double>(m, psiT.size());
  m->dinv = alloc_n<double>(m, dinv.size());
  m->bh = alloc_n<double>(m, (size_t)nxc * nyc * nb);
  m->bP = L >= 2 ? m->lv[L - 2].P : 1;
  m->bpart = alloc_n<double>(m, (size_t)m->bP * nb);
  m->xpart = alloc_n<double>(m, (size_t)nyc * nb);
  if (!m->phi || !m->phiT || !m->psi || !m->psiT || !m->dinv || !m->bh || !m->bpart || !m->xpart)
    return fail("coarsest-level buffers");
  hipError_t e = hipMemcpyAsync(m->phi, phi.data(), phi.size() * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(m->phiT, phiT.data(), phiT.size() * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(m->psi, psi.data(), psi.size() * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(m->psiT, psiT.data(), psiT.size() * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(m->dinv, dinv.data(), dinv.size() * 8, hipMemcpyHostToDevice, s);
  // the staging vectors above and the levels' upload arrays go out of scope
  const hipError_t es = hipStreamSynchronize(s);
  if (e != hipSuccess || es != hipSuccess) return fail("upload");
  p->mg = m;
  return PPE_OK;
}

}  // namespace ppe
