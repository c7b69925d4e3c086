// Per-grid setup: the 1D coefficient arrays of the finite-volume operator,
// built once per grid and reused by every solve (the paper builds its matrix
// and preconditioner once and reuses them at every time step, Sec. 2.5).
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "api_internal.hpp"
#include "mg_internal.hpp"

namespace ppe {

// Uploads the padded 1D coefficient arrays of a tensor grid (widths h, face
// factors g with g = 0 on the walls, centres) and fills c. The copies are
// ordered on stream s; the caller synchronises s before the host arrays go.
ppe_status coef_upload(int nx, int ny, const double* hx, const double* hy, const double* gx, const double* gy,
                       const double* xc, const double* yc, hipStream_t s, std::vector<double>& h64,
                       std::vector<float>& h32, void** dev, Coef* cout) {
  // Each array is stored with zero padding (kPadX columns on both sides,
  // kPadY0 rows before and kPadY1 after), so kernels may read indices just
  // outside the grid without bounds tests: hx[-1], gx[nx + 1], hy[ny + 80] ...
  const size_t lx = nx + 2 * kPadX, lgx = nx + 1 + 2 * kPadX;
  const size_t ly = ny + kPadY0 + kPadY1, lgy = ny + 1 + kPadY0 + kPadY1;
  const size_t n64 = lx + ly + lgx + lgy + nx + ny;
  h64.assign(n64, 0.0);
  double* hxp = h64.data();
  double* hyp = hxp + lx;
  double* gxp = hyp + ly;
  double* gyp = gxp + lgx;
  for (int i = 0; i < nx; ++i) hxp[kPadX + i] = hx[i];
  for (int j = 0; j < ny; ++j) hyp[kPadY0 + j] = hy[j];
  for (int k = 0; k <= nx; ++k) gxp[kPadX + k] = gx[k];
  for (int k = 0; k <= ny; ++k) gyp[kPadY0 + k] = gy[k];
  double* xcp = gyp + lgy;
  double* ycp = xcp + nx;
  for (int i = 0; i < nx; ++i) xcp[i] = xc[i];
  for (int j = 0; j < ny; ++j) ycp[j] = yc[j];
  h32.assign(h64.begin(), h64.end());
  const size_t bytes = n64 * (sizeof(double) + sizeof(float));
  *dev = dev_alloc(bytes);
  if (!*dev) return set_error(PPE_ERR_HIP, "device allocation of grid coefficients failed");
  double* d64 = (double*)*dev;
  float* d32 = (float*)(d64 + n64);
  if (hipMemcpyAsync(d64, h64.data(), n64 * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(d32, h32.data(), n64 * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess) {
    (void)hipStreamSynchronize(s);
    return set_error(PPE_ERR_HIP, "upload of grid coefficients failed");
  }
  Coef& c = *cout;
  c.nx = nx;
  c.ny = ny;
  c.hx64 = d64 + kPadX;
  c.hy64 = d64 + lx + kPadY0;
  c.gx64 = d64 + lx + ly + kPadX;
  c.gy64 = d64 + lx + ly + lgx + kPadY0;
  c.xc64 = d64 + lx + ly + lgx + lgy;
  c.yc64 = c.xc64 + nx;
  c.hx = d32 + kPadX;
  c.hy = d32 + lx + kPadY0;
  c.gx = d32 + lx + ly + kPadX;
  c.gy = d32 + lx + ly + lgx + kPadY0;
  return PPE_OK;
}

ppe_status problem_upload(ppe_problem* p, hipStream_t s) {
  const int nx = p->nx, ny = p->ny;
  // Face conductance factors: 1/(centre distance) on interior faces, 0 on walls.
  std::vector<double> gx(nx + 1, 0.0), gy(ny + 1, 0.0);
  for (int k = 1; k < nx; ++k) gx[k] = 1.0 / (p->xc[k] - p->xc[k - 1]);
  for (int k = 1; k < ny; ++k) gy[k] = 1.0 / (p->yc[k] - p->yc[k - 1]);
  std::vector<double> h64;
  std::vector<float> h32;
  ppe_status up = coef_upload(nx, ny, p->hx.data(), p->hy.data(), gx.data(), gy.data(), p->xc.data(),
                              p->yc.data(), s, h64, h32, &p->dev_coef, &p->coef);
  if (up != PPE_OK) return up;
  ppe_status st = PPE_OK;
  std::vector<float> fl, dinv;
  if (p->mask_mode == PPE_MASK_SOLID) {
    // fluid flags and the inverse diagonal of the solid-mask operator (FP64, rounded once)
    const size_t N = (size_t)nx * ny;
    fl.resize(N);
    dinv.resize(N);
    int64_t nf = 0;
    auto isf = [&](int i, int j) { return p->mask[(size_t)j * nx + i] == 0; };
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const size_t c = (size_t)j * nx + i;
        fl[c] = isf(i, j) ? 1.f : 0.f;
        if (!isf(i, j)) {
          dinv[c] = 1.f;
          continue;
        }
        ++nf;
        double d = 0.0;
        if (i > 0 && isf(i - 1, j)) d += p->hy[j] * gx[i];
        if (i + 1 < nx && isf(i + 1, j)) d += p->hy[j] * gx[i + 1];
        if (j > 0 && isf(i, j - 1)) d += p->hx[i] * gy[j];
        if (j + 1 < ny && isf(i, j + 1)) d += p->hx[i] * gy[j + 1];
        dinv[c] = d > 0.0 ? (float)(1.0 / d) : 0.f;  // an isolated fluid cell has no equation
      }
    p->d_solid = (float*)dev_alloc(sizeof(float) * 2 * N);
    if (!p->d_solid) st = set_error(PPE_ERR_HIP, "device allocation of the solid-mask arrays failed");
    else if (hipMemcpyAsync(p->d_solid, fl.data(), sizeof(float) * N, hipMemcpyHostToDevice, s) != hipSuccess ||
             hipMemcpyAsync(p->d_solid + N, dinv.data(), sizeof(float) * N, hipMemcpyHostToDevice, s) != hipSuccess)
      st = set_error(PPE_ERR_HIP, "upload of the solid-mask arrays failed");
    p->coef.fl = p->d_solid;
    p->coef.dinv = p->d_solid + N;
    p->coef.nfluid = nf;
  }
  if (st == PPE_OK && !p->mask.empty()) {
    p->d_mask = (uint8_t*)dev_alloc(p->mask.size());
    if (!p->d_mask) st = set_error(PPE_ERR_HIP, "device allocation of the mask failed");
    else if (hipMemcpyAsync(p->d_mask, p->mask.data(), p->mask.size(), hipMemcpyHostToDevice, s) != hipSuccess)
      st = set_error(PPE_ERR_HIP, "upload of the mask failed");
  }
  // the host staging vectors go out of scope: the copies must have finished
  if (hipStreamSynchronize(s) != hipSuccess && st == PPE_OK)
    st = set_error(PPE_ERR_HIP, "grid upload: stream sync failed");
  return st;
}

void problem_release(ppe_problem* p) {
  net_cache_free(p->net_cache);
  p->net_cache = nullptr;
  mg_free(p->mg);
  p->mg = nullptr;
  dev_free(p->dev_coef);
  p->dev_coef = nullptr;
  dev_free(p->d_mask);
  p->d_mask = nullptr;
  dev_free(p->d_solid);
  p->d_solid = nullptr;
  dev_free(p->d_icq);
  dev_free(p->d_icz);
  p->d_icq = p->d_icz = nullptr;
  p->ic_nb = 0;
}

}  // namespace ppe
