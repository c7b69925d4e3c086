// Training-data generator on the device: the fabricated right-hand sides that
// stand in for the Lanczos-Ritz vectors of Eqs. 14-16 (HIP, gfx950).
//
// Definition (shared with nothing: the test reference implements it
// separately):
//   * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011), key = (seed mod
//     2^32, seed div 2^32), counter = (draw index d, sample s, step mod 2^32,
//     step div 2^32); an output word x maps to u = ((x >> 8) + 1/2) 2^-24;
//   * sample s, draw 0: length scale l = exp(ln l_lo + u0 (ln l_hi - ln l_lo));
//   * feature f < J, draw 1 + f: w = sqrt(-2 ln u0) (cos 2 pi u1, sin 2 pi u1) / l,
//     phase phi = 2 pi u2;
//   * random Fourier features (Rahimi & Recht, 2007) for the squared-
//     exponential covariance exp(-|d|^2 / (2 l^2)):
//     g(x, y) = sqrt(2/J) sum_f cos(w_x x + w_y y + phi), at the cell centres;
//   * R = (cell area) g, minus its mean, divided by its RMS (FP32 output).
// Evaluation: cos(a + b) = cos a cos b - sin a sin b with a = w_x x + phi and
// b = w_y y, so a 64 x 64 tile needs the 1D tables of its 64 columns and 64
// rows per feature (staged in LDS, 16 features at a time), about 16 FP64
// sincos per cell instead of J. Sums are FP64 with fixed-order reductions.
#include <hip/hip_runtime.h>

#include <cmath>

#include "api_internal.hpp"
#include "rng.hpp"

namespace ppe {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr int kGenTile = 64, kGenChunk = 16;

struct GenKey {
  uint32_t k0, k1, st0, st1;
  double ln_lo, ln_hi;
  int J;
};

// Features of every sample: feat[s][f] = (w_x, w_y, phi, l).
__global__ __launch_bounds__(256) void k_grf_features(GenKey g, double4* __restrict__ feat) {
  const int s = blockIdx.x;
  const uint4 c0 = philox4x32_10(make_uint4(0u, (uint32_t)s, g.st0, g.st1), g.k0, g.k1);
  const double ell = exp(g.ln_lo + unit01(c0.x) * (g.ln_hi - g.ln_lo));
  for (int f = threadIdx.x; f < g.J; f += blockDim.x) {
    const uint4 c = philox4x32_10(make_uint4((uint32_t)(1 + f), (uint32_t)s, g.st0, g.st1), g.k0, g.k1);
    const double rad = sqrt(-2.0 * log(unit01(c.x)));
    double sn, cs;
    sincos(kTwoPi * unit01(c.y), &sn, &cs);
    feat[(size_t)s * g.J + f] = make_double4(rad * cs / ell, rad * sn / ell, kTwoPi * unit01(c.z), ell);
  }
}

// raw = (cell area) g on 64 x 64 tiles; per-tile sums of raw and raw^2.
__global__ __launch_bounds__(256) void k_grf_field(const Coef* __restrict__ coefs, int J,
                                                   const double4* __restrict__ feat, double* __restrict__ raw,
                                                   double* __restrict__ part) {
  __shared__ double cxs[kGenChunk][kGenTile], sxs[kGenChunk][kGenTile];
  __shared__ double cys[kGenChunk][kGenTile], sys[kGenChunk][kGenTile];
  __shared__ double red[2][kWaves];
  const int s = blockIdx.z;
  const Coef c = coefs[s];
  const int nx = c.nx, ny = c.ny;
  const int i0 = blockIdx.x * kGenTile, j0 = blockIdx.y * kGenTile;
  const int t = threadIdx.x, ci = t & (kGenTile - 1), rq = t / kGenTile;
  const double4* fs = feat + (size_t)s * J;
  double acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = 0.0;
  for (int f0 = 0; f0 < J; f0 += kGenChunk) {
    __syncthreads();
    for (int q = t; q < kGenChunk * kGenTile; q += kBlock) {
      const int ff = q / kGenTile, e = q % kGenTile, f = f0 + ff;
      double ca = 0.0, sa = 0.0, cb = 0.0, sb = 0.0;
      if (f < J) {
        const double4 w = fs[f];
        sincos(w.x * c.xc64[min(i0 + e, nx - 1)] + w.z, &sa, &ca);
        sincos(w.y * c.yc64[min(j0 + e, ny - 1)], &sb, &cb);
      }
      cxs[ff][e] = ca;
      sxs[ff][e] = sa;
      cys[ff][e] = cb;
      sys[ff][e] = sb;
    }
    __syncthreads();
#pragma unroll 4
    for (int ff = 0; ff < kGenChunk; ++ff) {
      const double cx = cxs[ff][ci], sx = sxs[ff][ci];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int e = rq + kWaves * k;
        acc[k] += cx * cys[ff][e] - sx * sys[ff][e];
      }
    }
  }
  const double scale = sqrt(2.0 / (double)J);
  const int i = i0 + ci;
  double s1 = 0.0, s2 = 0.0;
  if (i < nx) {
    const double hx = c.hx64[i];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int j = j0 + rq + kWaves * k;
      if (j < ny) {
        const double v = hx * c.hy64[j] * (scale * acc[k]);
        raw[(size_t)s * nx * ny + (size_t)j * nx + i] = v;
        s1 += v;
        s2 += v * v;
      }
    }
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if ((t & (kWave - 1)) == 0) {
    red[0][t / kWave] = s1;
    red[1][t / kWave] = s2;
  }
  __syncthreads();
  if (t == 0) {
    const int P = gridDim.x * gridDim.y, b = blockIdx.y * gridDim.x + blockIdx.x;
    double* ps = part + (size_t)s * 2 * P;
    ps[b] = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
    ps[P + b] = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
  }
}

// R = (raw - mean) / rms in FP32; every workgroup re-reduces its sample's
// tile sums in the same order.
__global__ __launch_bounds__(256) void k_grf_normalise(int64_t N, int P, const double* __restrict__ raw,
                                                       const double* __restrict__ part, float* __restrict__ R) {
  __shared__ double lds[kWaves];
  const int s = blockIdx.y;
  const double* ps = part + (size_t)s * 2 * P;
  const double sum = reduce_partials(ps, P, lds);
  const double sq = reduce_partials(ps + P, P, lds);
  const double mean = sum / (double)N;
  const double rms = sqrt(sq / (double)N - mean * mean);
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k < N) R[(size_t)s * N + k] = (float)((raw[(size_t)s * N + k] - mean) / rms);
}

ppe_status gen_ensure(GenWs& w, int nb, int64_t N, int J, int P) {
  if (w.nb >= nb && w.N >= N && w.J >= J && w.P >= P) return PPE_OK;
  gen_free(w);
  w.feat = dev_alloc(sizeof(double4) * (size_t)nb * J);
  w.raw = (double*)dev_alloc(sizeof(double) * (size_t)nb * N);
  w.part = (double*)dev_alloc(sizeof(double) * 2 * (size_t)nb * P);
  w.coefs = (Coef*)dev_alloc(sizeof(Coef) * nb);
  if (!w.feat || !w.raw || !w.part || !w.coefs) {
    gen_free(w);
    return set_error(PPE_ERR_HIP, "allocation of the data-generator workspace failed");
  }
  w.nb = nb;
  w.N = N;
  w.J = J;
  w.P = P;
  return PPE_OK;
}

void gen_free(GenWs& w) {
  dev_free(w.feat);
  dev_free(w.raw);
  dev_free(w.part);
  dev_free(w.coefs);
  w = GenWs{};
}

ppe_status check_gen_opts(const ppe_train_opts& o) {
  if (!(o.grf_len_lo > 0.f) || !(o.grf_len_hi >= o.grf_len_lo) || !std::isfinite(o.grf_len_hi))
    return set_error(PPE_ERR_INVALID_ARG, "need 0 < grf_len_lo <= grf_len_hi (finite)");
  if (o.grf_features < 1 || o.grf_features > 65536)
    return set_error(PPE_ERR_INVALID_ARG, "grf_features must lie in [1, 65536]");
  if (o.step < 0) return set_error(PPE_ERR_INVALID_ARG, "step must be >= 0");
  return PPE_OK;
}

ppe_status generate_rhs(GenWs& w, int nb, ppe_problem* const* probs, const ppe_train_opts& o, float* R,
                        hipStream_t s) {
  const int nx = probs[0]->nx, ny = probs[0]->ny;
  const int64_t N = (int64_t)nx * ny;
  const int J = o.grf_features;
  const dim3 tiles((nx + kGenTile - 1) / kGenTile, (ny + kGenTile - 1) / kGenTile, nb);
  const int P = (int)(tiles.x * tiles.y);
  ppe_status st = gen_ensure(w, nb, N, J, P);
  if (st != PPE_OK) return st;
  std::vector<Coef> cs(nb);
  for (int i = 0; i < nb; ++i) cs[i] = probs[i]->coef;
  if (hipMemcpyAsync(w.coefs, cs.data(), sizeof(Coef) * nb, hipMemcpyHostToDevice, s) != hipSuccess)
    return set_error(PPE_ERR_HIP, "upload of the generator's grid descriptors failed");
  GenKey g;
  g.k0 = (uint32_t)(o.seed & 0xffffffffu);
  g.k1 = (uint32_t)(o.seed >> 32);
  g.st0 = (uint32_t)((uint64_t)o.step & 0xffffffffu);
  g.st1 = (uint32_t)((uint64_t)o.step >> 32);
  g.ln_lo = std::log((double)o.grf_len_lo);
  g.ln_hi = std::log((double)o.grf_len_hi);
  g.J = J;
  k_grf_features<<<nb, kBlock, 0, s>>>(g, (double4*)w.feat);
  k_grf_field<<<tiles, kBlock, 0, s>>>(w.coefs, J, (const double4*)w.feat, w.raw, w.part);
  k_grf_normalise<<<dim3((unsigned)((N + kBlock - 1) / kBlock), nb), kBlock, 0, s>>>(N, P, w.raw, w.part, R);
  if (hipGetLastError() != hipSuccess) return set_error(PPE_ERR_HIP, "data-generator launch failed");
  // the descriptor vector is released on return: finish its copy first
  if (hipStreamSynchronize(s) != hipSuccess) return set_error(PPE_ERR_HIP, "data-generator stream sync failed");
  return PPE_OK;
}

}  // namespace ppe

using namespace ppe;

// Grid of a fabricated training system, drawn on the host (2 Philox blocks
// and O(nx + ny + nx ny) arithmetic: no kernel launch pays for itself). The
// draws use counter indices past those of the source fields.
namespace {
constexpr uint32_t kGridDraw = 0xFFFFFF00u;

uint4 philox_host(uint4 c, uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

double unit01_host(uint32_t x) { return ((double)(x >> 8) + 0.5) * 0x1p-24; }

// tanh-stretched axis of n cells on [0, 1]: faces, then centres and widths
void tanh_axis(int n, double beta, double* c, double* h) {
  const double tb = std::tanh(beta);
  double f0 = 0.0;
  for (int i = 0; i < n; ++i) {
    const double f1 = i + 1 == n ? 1.0 : 0.5 * (1.0 + std::tanh(beta * (2.0 * (i + 1) / n - 1.0)) / tb);
    c[i] = 0.5 * (f0 + f1);
    h[i] = f1 - f0;
    f0 = f1;
  }
}
}  // namespace

extern "C" ppe_status ppe_generate_grid(int32_t nx, int32_t ny, uint64_t seed, uint64_t step, int32_t sample,
                                        double* xc, double* yc, double* hx, double* hy, uint8_t* mask,
                                        double* params) {
  if (nx < 2 || ny < 2 || (int64_t)nx * ny > ((int64_t)1 << 28))
    return set_error(PPE_ERR_INVALID_ARG, "grid %d x %d outside [2, 2^28 cells]", nx, ny);
  if (sample < 0) return set_error(PPE_ERR_INVALID_ARG, "sample < 0");
  if (!xc || !yc || !hx || !hy) return set_error(PPE_ERR_INVALID_ARG, "xc, yc, hx or hy is NULL");
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  auto draw = [&](uint32_t d) {
    return philox_host(make_uint4(d, (uint32_t)sample, (uint32_t)step, (uint32_t)(step >> 32)), k0, k1);
  };
  const uint4 a = draw(kGridDraw), b = draw(kGridDraw + 1);
  const double bx = 1.0 + 1.5 * unit01_host(a.x), by = 1.0 + 1.5 * unit01_host(a.y);
  const double cx = 0.25 + 0.5 * unit01_host(a.z), cy = 0.25 + 0.5 * unit01_host(a.w);
  const double ea = 0.05 + 0.1 * unit01_host(b.x), eb = 0.05 + 0.1 * unit01_host(b.y);
  const double th = M_PI * unit01_host(b.z);
  tanh_axis(nx, bx, xc, hx);
  tanh_axis(ny, by, yc, hy);
  if (mask) {
    const double ct = std::cos(th), st = std::sin(th);
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const double dx = xc[i] - cx, dy = yc[j] - cy;
        const double u = (dx * ct + dy * st) / ea, v = (dy * ct - dx * st) / eb;
        mask[(int64_t)j * nx + i] = u * u + v * v <= 1.0;
      }
  }
  if (params) {
    const double pv[7] = {bx, by, cx, cy, ea, eb, th};
    for (int k = 0; k < 7; ++k) params[k] = pv[k];
  }
  return PPE_OK;
}

extern "C" ppe_status ppe_generate_rhs(int32_t nb, ppe_problem* const* problems, const ppe_train_opts* opts, float* R,
                                       hipStream_t s) {
  if (nb < 0 || (nb > 0 && (!problems || !R)) || !opts) return set_error(PPE_ERR_INVALID_ARG, "bad arguments");
  if (nb == 0) return PPE_OK;
  if (nb > 65535) return set_error(PPE_ERR_INVALID_ARG, "nb > 65535");
  for (int i = 0; i < nb; ++i) {
    if (!problems[i]) return set_error(PPE_ERR_INVALID_ARG, "problems[%d] is NULL", i);
    if (problems[i]->mask_mode == PPE_MASK_SOLID) return reject_solid(problems[i], "ppe_generate_rhs");
    if (problems[i]->nx != problems[0]->nx || problems[i]->ny != problems[0]->ny)
      return set_error(PPE_ERR_SHAPE, "all grids of a batch must have one size");
  }
  ppe_status st = check_gen_opts(*opts);
  if (st != PPE_OK) return st;
  static thread_local GenWs ws;
  return generate_rhs(ws, nb, problems, *opts, R, s);
}
