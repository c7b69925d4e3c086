// Lanczos-Ritz training vectors (Sec. 2.3, Eqs. 14-16) on one grid.
//
// Lanczos on the finite-volume operator A from a start vector v0 (projected
// onto zero mean, normalised): m steps in FP64 on the device, each
//   w = A v_j;  w -= B (B^T w), twice (classical Gram-Schmidt applied twice)
// with B = [1/sqrt(N), v_0 .. v_j] the constant null vector and every earlier
// Lanczos vector, so that the basis stays orthonormal over long runs;
//   alpha_j = v_j . A v_j (the coefficient of v_j in the two passes),
//   beta_j = |w|, v_{j+1} = w / beta_j.
// The basis lives in device memory as rows 1..m of V (row 0 is the null
// vector). T_m = tridiag(beta, alpha, beta) (Eq. 14) is diagonalised on the
// host by implicit symmetric QR steps with Wilkinson shifts (Golub and Van
// Loan, Matrix Computations, Sec. 8.3), giving ascending Ritz values theta
// and T_m = U diag(theta) U^T; U goes back to the device.
//
// A batch of training vectors R^i = Q c^i / |Q c^i| (Eqs. 15-16, Q = V_m U)
// is formed without Q: y = U c on the device, then R = V_m y, then the norm
// (FP64, fixed order) and the FP32 output. The normal draws c_j^i come from
// Philox4x32-10 with key = seed and counter (j, i + 2^31, step lo, step hi)
// by Box-Muller, times 9 for j <= b m.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "api_internal.hpp"
#include "rng.hpp"

struct ppe_ritz {
  int nx = 0, ny = 0;
  int64_t N = 0;
  int m = 0;                       // Lanczos vectors kept
  double* d_V = nullptr;           // [m + 1][N], row 0 = 1 / sqrt(N)
  double* d_U = nullptr;           // [m][m], U[k][j] = component k of eigenvector j
  std::vector<double> alpha, beta, theta;
};

namespace ppe {

#define HIPCHK(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return set_error(PPE_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

constexpr int kRB = 256;        // threads per block
constexpr int kNormBlocks = 64; // partial sums of a norm

// c[k] = B[k] . w for the rows k < nrows of B ([nrows][N]); one block per row,
// fixed-order block sum.
__global__ __launch_bounds__(kRB) void k_rows_dot(const double* __restrict__ B, int64_t N,
                                                 const double* __restrict__ w, double* __restrict__ c) {
  __shared__ double lds[kRB / kWave];
  const double* b = B + (size_t)blockIdx.x * N;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += kRB) s += b[i] * w[i];
  s = block_sum(s, lds);
  if (threadIdx.x == 0) c[blockIdx.x] = s;
}

// w -= B^T c over the rows k < nrows, and acc[col] += c[col] (the coefficient
// of one chosen row, accumulated over the passes) by the first thread.
__global__ __launch_bounds__(kRB) void k_rows_sub(const double* __restrict__ B, int nrows, int64_t N,
                                                 const double* __restrict__ c, double* __restrict__ w, int col,
                                                 double* __restrict__ acc) {
  const int64_t i = (int64_t)blockIdx.x * kRB + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) acc[0] += c[col];
  if (i >= N) return;
  double v = w[i];
  for (int k = 0; k < nrows; ++k) v -= B[(size_t)k * N + i] * c[k];
  w[i] = v;
}

// Partial sums of x^2 (kNormBlocks blocks, fixed order).
__global__ __launch_bounds__(kRB) void k_sumsq64(const double* __restrict__ x, int64_t N, double* __restrict__ part) {
  __shared__ double lds[kRB / kWave];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kRB) s += x[i] * x[i];
  s = block_sum(s, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out = w / |w| with |w| from the partials (reduced alike in every block);
// the norm is stored in *beta. Below `tiny` the Krylov space is exhausted:
// out = 0 and beta = 0.
__global__ __launch_bounds__(kRB) void k_next_vector(const double* __restrict__ w, int64_t N,
                                                    const double* __restrict__ part, double tiny,
                                                    double* __restrict__ out, double* __restrict__ beta) {
  __shared__ double lds[kRB / kWave];
  const double nrm = sqrt(reduce_partials(part, kNormBlocks, lds));
  const bool ok = nrm > tiny;
  if (blockIdx.x == 0 && threadIdx.x == 0) *beta = ok ? nrm : 0.0;
  const double inv = ok ? 1.0 / nrm : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kRB) out[i] = w[i] * inv;
}

__global__ void k_fill(double* x, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * kRB + threadIdx.x;
  if (i < n) x[i] = v;
}

// c[s][j] of Eq. 16 for samples s < nb.
__global__ __launch_bounds__(kRB) void k_ritz_coef(int m, int nb, int jmax, uint32_t k0, uint32_t k1, uint32_t st0,
                                                  uint32_t st1, double* __restrict__ c) {
  const int64_t t = (int64_t)blockIdx.x * kRB + threadIdx.x;
  if (t >= (int64_t)m * nb) return;
  const int s = (int)(t / m), j = (int)(t % m);
  const uint4 r = philox4x32_10(make_uint4((uint32_t)j, (uint32_t)s | 0x80000000u, st0, st1), k0, k1);
  const double g = sqrt(-2.0 * log(unit01(r.x))) * cos(6.283185307179586476925286766559 * unit01(r.y));
  c[t] = j <= jmax ? 9.0 * g : g;
}

// y[s][k] = sum_j U[k][j] c[s][j]: one block per (k, s), fixed-order block sum.
__global__ __launch_bounds__(kRB) void k_u_times_c(const double* __restrict__ U, int m, const double* __restrict__ c,
                                                  double* __restrict__ y) {
  __shared__ double lds[kRB / kWave];
  const int k = blockIdx.x, s = blockIdx.y;
  const double* u = U + (size_t)k * m;
  const double* cs = c + (size_t)s * m;
  double v = 0.0;
  for (int j = threadIdx.x; j < m; j += kRB) v += u[j] * cs[j];
  v = block_sum(v, lds);
  if (threadIdx.x == 0) y[(size_t)s * m + k] = v;
}

// r[s][i] = sum_k V[k + 1][i] y[s][k] (rows 1..m of V).
__global__ __launch_bounds__(kRB) void k_v_times_y(const double* __restrict__ V, int m, int64_t N,
                                                  const double* __restrict__ y, double* __restrict__ r) {
  const int s = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * kRB + threadIdx.x;
  if (i >= N) return;
  const double* ys = y + (size_t)s * m;
  double v = 0.0;
  for (int k = 0; k < m; ++k) v += V[(size_t)(k + 1) * N + i] * ys[k];
  r[(size_t)s * N + i] = v;
}

// R[s] = r[s] / |r[s]| in FP32; |r[s]|^2 from kNormBlocks partials per sample.
__global__ __launch_bounds__(kRB) void k_sumsq64_batch(const double* __restrict__ r, int64_t N,
                                                      double* __restrict__ part) {
  __shared__ double lds[kRB / kWave];
  const double* x = r + (size_t)blockIdx.y * N;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kRB) s += x[i] * x[i];
  s = block_sum(s, lds);
  if (threadIdx.x == 0) part[(size_t)blockIdx.y * kNormBlocks + blockIdx.x] = s;
}

__global__ __launch_bounds__(kRB) void k_normalise(const double* __restrict__ r, int64_t N,
                                                  const double* __restrict__ part, double scale,
                                                  float* __restrict__ R) {
  __shared__ double lds[kRB / kWave];
  const int s = blockIdx.y;
  const double nrm = sqrt(reduce_partials(part + (size_t)s * kNormBlocks, kNormBlocks, lds));
  const double inv = nrm > 0.0 ? scale / nrm : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kRB)
    R[(size_t)s * N + i] = (float)(r[(size_t)s * N + i] * inv);
}

static unsigned blocks_for(int64_t n) { return (unsigned)((n + kRB - 1) / kRB); }

// ---------------------------------------------------------------------------
// Host: eigen-decomposition of a symmetric tridiagonal matrix by implicit QR
// steps with Wilkinson shifts (Golub and Van Loan, Sec. 8.3). a: diagonal
// (n), b: off-diagonal (n - 1); both are overwritten and the eigenvalues are
// returned in a (in the order the iteration leaves them). Each step chases a
// bulge down the unreduced block [p, q] with Givens rotations G acting on
// coordinates k, k+1 (G_kk = G_k+1,k+1 = c, G_k,k+1 = s, G_k+1,k = -s),
// T <- G^T T G; the eigenvector matrix is Z = G_1 G_2 ... (Z <- Z G for
// each rotation in turn). The rotations are recorded, one sweep (QR step)
// at a time: sweeps[t] = {first rotation, p, q}, rotation r acting on
// coordinates p + (r - first), p + (r - first) + 1.
struct QrSweeps {
  std::vector<int64_t> first;
  std::vector<int> p, q;
  std::vector<double> c, s;
};

static bool tridiag_qr(int n, std::vector<double>& a, std::vector<double>& b, QrSweeps& sw) {
  sw = QrSweeps{};
  const double eps = 2.220446049250313e-16;
  auto small = [&](int k) { return std::fabs(b[k]) <= eps * (std::fabs(a[k]) + std::fabs(a[k + 1])); };
  int q = n - 1;
  int64_t steps = 0;
  while (q > 0) {
    if (small(q - 1)) {
      b[q - 1] = 0.0;
      --q;
      continue;
    }
    int p = q - 1;
    while (p > 0 && !small(p - 1)) --p;
    if (p > 0) b[p - 1] = 0.0;
    if (++steps > 60LL * n + 100) return false;
    sw.first.push_back((int64_t)sw.c.size());
    sw.p.push_back(p);
    sw.q.push_back(q);
    // Wilkinson shift from the trailing 2 x 2 block of [p, q]
    const double d = 0.5 * (a[q - 1] - a[q]);
    const double bq = b[q - 1];
    const double mu = a[q] - bq * bq / (d + (d >= 0.0 ? 1.0 : -1.0) * std::hypot(d, bq));
    double x = a[p] - mu, z = b[p];
    for (int k = p; k < q; ++k) {
      const double r = std::hypot(x, z);
      const double c = r > 0.0 ? x / r : 1.0, s = r > 0.0 ? -z / r : 0.0;
      if (k > p) b[k - 1] = r;
      const double ak = a[k], ak1 = a[k + 1], bk = b[k];
      a[k] = ak * c * c - 2.0 * bk * c * s + ak1 * s * s;
      a[k + 1] = ak * s * s + 2.0 * bk * c * s + ak1 * c * c;
      b[k] = (ak - ak1) * c * s + bk * (c * c - s * s);
      if (k + 1 < q) {
        const double g = b[k + 1];
        z = -s * g;
        b[k + 1] = c * g;
        x = b[k];
      }
      sw.c.push_back(c);
      sw.s.push_back(s);
    }
  }
  return true;
}

// Ascending order of the eigenvalues in a (a stable sort of the indices).
static std::vector<int> ascending(const std::vector<double>& a) {
  std::vector<int> ord(a.size());
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int i, int j) { return a[i] < a[j]; });
  return ord;
}

// Z <- Z G for every recorded rotation, on the host (Z row-major n x n,
// starting from the identity), then the columns in ascending order of the
// eigenvalues and each signed so that its first component (for T_m, the
// component along the start vector v_0) is not negative.
static void eigvecs_host(int n, const std::vector<double>& a, const QrSweeps& sw, std::vector<double>& U) {
  std::vector<double> Z((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
  for (size_t t = 0; t < sw.first.size(); ++t)
    for (int k = sw.p[t]; k < sw.q[t]; ++k) {
      const double c = sw.c[sw.first[t] + (k - sw.p[t])], s = sw.s[sw.first[t] + (k - sw.p[t])];
      for (int i = 0; i < n; ++i) {
        double* zi = &Z[(size_t)i * n];
        const double u = zi[k], v = zi[k + 1];
        zi[k] = c * u - s * v;
        zi[k + 1] = s * u + c * v;
      }
    }
  const std::vector<int> ord = ascending(a);
  U.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    const double sg = Z[ord[j]] < 0.0 ? -1.0 : 1.0;
    for (int i = 0; i < n; ++i) U[(size_t)i * n + j] = sg * Z[(size_t)i * n + ord[j]];
  }
}

// The same on the device. Zc is column-major (Zc[k][i] = component i of
// column k), so one thread per component i reads and writes coalesced rows.
// A thread walks the sweeps in order; within a sweep the coordinates rise by
// one per rotation, so the column just rotated into position k + 1 is kept
// in a register for the next rotation, and the next kRotAhead columns are
// loaded before they are used (none of them has been written in this sweep).
constexpr int kRotAhead = 16;
__global__ __launch_bounds__(kRB) void k_apply_sweeps(double* __restrict__ Zc, int n, int nsweeps,
                                                     const int* __restrict__ sp, const int* __restrict__ sq,
                                                     const int64_t* __restrict__ sfirst,
                                                     const double* __restrict__ rc, const double* __restrict__ rs) {
  const int i = blockIdx.x * kRB + threadIdx.x;
  if (i >= n) return;
  for (int t = 0; t < nsweeps; ++t) {
    const int p = sp[t], q = sq[t];
    const double* c = rc + sfirst[t];
    const double* s = rs + sfirst[t];
    double u = Zc[(size_t)p * n + i];
    for (int k0 = p; k0 < q; k0 += kRotAhead) {
      double v[kRotAhead];
#pragma unroll
      for (int r = 0; r < kRotAhead; ++r) v[r] = (k0 + r < q) ? Zc[(size_t)(k0 + r + 1) * n + i] : 0.0;
#pragma unroll
      for (int r = 0; r < kRotAhead; ++r) {
        const int k = k0 + r;
        if (k >= q) break;
        const double cc = c[k - p], ss = s[k - p];
        Zc[(size_t)k * n + i] = cc * u - ss * v[r];
        u = ss * u + cc * v[r];
      }
    }
    Zc[(size_t)q * n + i] = u;
  }
}

// U[i][j] = sign_j Zc[ord[j]][i] (row-major U, the layout the Ritz kernels read).
__global__ __launch_bounds__(kRB) void k_order_eigvecs(const double* __restrict__ Zc, int n,
                                                      const int* __restrict__ ord, const double* __restrict__ sign,
                                                      double* __restrict__ U) {
  const int64_t t = (int64_t)blockIdx.x * kRB + threadIdx.x;
  if (t >= (int64_t)n * n) return;
  const int i = (int)(t / n), j = (int)(t % n);
  U[t] = sign[j] * Zc[(size_t)ord[j] * n + i];
}

// Eigenvectors of the recorded sweeps on the device, into d_U (n x n,
// row-major), sweeps uploaded in chunks of at most kChunk rotations.
static ppe_status eigvecs_device(int n, const std::vector<double>& a, const QrSweeps& sw, double* d_U,
                                 hipStream_t st) {
  constexpr int64_t kChunk = (int64_t)1 << 22;
  const int64_t nrot = (int64_t)sw.c.size();
  const int64_t nsw = (int64_t)sw.first.size();
  double* Zc = (double*)dev_alloc(sizeof(double) * (size_t)n * n);
  double *d_c = (double*)dev_alloc(sizeof(double) * (size_t)std::min<int64_t>(std::max<int64_t>(nrot, 1), kChunk + n));
  double *d_s = (double*)dev_alloc(sizeof(double) * (size_t)std::min<int64_t>(std::max<int64_t>(nrot, 1), kChunk + n));
  int* d_p = (int*)dev_alloc(sizeof(int) * (size_t)std::max<int64_t>(nsw, 1));
  int* d_q = (int*)dev_alloc(sizeof(int) * (size_t)std::max<int64_t>(nsw, 1));
  int64_t* d_f = (int64_t*)dev_alloc(sizeof(int64_t) * (size_t)std::max<int64_t>(nsw, 1));
  int* d_ord = (int*)dev_alloc(sizeof(int) * n);
  double* d_sg = (double*)dev_alloc(sizeof(double) * n);
  auto done = [&](ppe_status st_) {
    dev_free(Zc); dev_free(d_c); dev_free(d_s); dev_free(d_p); dev_free(d_q); dev_free(d_f); dev_free(d_ord);
    dev_free(d_sg);
    return st_;
  };
  if (!Zc || !d_c || !d_s || !d_p || !d_q || !d_f || !d_ord || !d_sg)
    return done(set_error(PPE_ERR_HIP, "allocation for the Ritz eigenvectors failed"));
  // identity
  {
    std::vector<double> I((size_t)n * n, 0.0);
    for (int k = 0; k < n; ++k) I[(size_t)k * n + k] = 1.0;
    if (hipMemcpyAsync(Zc, I.data(), sizeof(double) * (size_t)n * n, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return done(set_error(PPE_ERR_HIP, "upload for the Ritz eigenvectors failed"));
  }
  std::vector<int64_t> rel(nsw);
  int64_t t0 = 0;
  while (t0 < nsw) {
    // sweeps t0 .. t1-1, at most kChunk rotations (a sweep has at most n - 1)
    int64_t t1 = t0;
    const int64_t r0 = sw.first[t0];
    while (t1 < nsw && (t1 == t0 || (t1 + 1 < nsw ? sw.first[t1 + 1] : nrot) - r0 <= kChunk)) ++t1;
    const int64_t r1 = t1 < nsw ? sw.first[t1] : nrot;
    for (int64_t t = t0; t < t1; ++t) rel[t] = sw.first[t] - r0;
    const size_t nr = (size_t)(r1 - r0), ns = (size_t)(t1 - t0);
    if (hipMemcpyAsync(d_c, sw.c.data() + r0, sizeof(double) * nr, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(d_s, sw.s.data() + r0, sizeof(double) * nr, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(d_p, sw.p.data() + t0, sizeof(int) * ns, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(d_q, sw.q.data() + t0, sizeof(int) * ns, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(d_f, rel.data() + t0, sizeof(int64_t) * ns, hipMemcpyHostToDevice, st) != hipSuccess)
      return done(set_error(PPE_ERR_HIP, "upload of the QR rotations failed"));
    k_apply_sweeps<<<blocks_for(n), kRB, 0, st>>>(Zc, n, (int)ns, d_p, d_q, d_f, d_c, d_s);
    // the host arrays of the next chunk overwrite these buffers
    if (hipStreamSynchronize(st) != hipSuccess) return done(set_error(PPE_ERR_HIP, "applying the QR rotations failed"));
    t0 = t1;
  }
  // order and signs: the first component of column k is Zc[k][0]
  std::vector<double> first(n);
  if (hipMemcpy2DAsync(first.data(), sizeof(double), Zc, sizeof(double) * (size_t)n, sizeof(double), n,
                       hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return done(set_error(PPE_ERR_HIP, "download of the eigenvector signs failed"));
  const std::vector<int> ord = ascending(a);
  std::vector<double> sg(n);
  for (int j = 0; j < n; ++j) sg[j] = first[ord[j]] < 0.0 ? -1.0 : 1.0;
  if (hipMemcpyAsync(d_ord, ord.data(), sizeof(int) * n, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(d_sg, sg.data(), sizeof(double) * n, hipMemcpyHostToDevice, st) != hipSuccess)
    return done(set_error(PPE_ERR_HIP, "upload of the eigenvector order failed"));
  k_order_eigvecs<<<blocks_for((int64_t)n * n), kRB, 0, st>>>(Zc, n, d_ord, d_sg, d_U);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
    return done(set_error(PPE_ERR_HIP, "ordering the Ritz eigenvectors failed"));
  return done(PPE_OK);
}

}  // namespace ppe

using namespace ppe;

extern "C" ppe_status ppe_tridiag_eigh(int32_t n, const double* alpha, const double* beta, double* theta, double* U) {
  if (n < 1 || !alpha || (n > 1 && !beta) || !theta) return set_error(PPE_ERR_INVALID_ARG, "bad arguments");
  std::vector<double> a(alpha, alpha + n), b(n > 1 ? n - 1 : 0), Z;
  if (n > 1) std::copy(beta, beta + n - 1, b.begin());
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(a[i]) || (i + 1 < n && !std::isfinite(b[i])))
      return set_error(PPE_ERR_NONFINITE, "non-finite tridiagonal entry");
  QrSweeps sw;
  if (!tridiag_qr(n, a, b, sw)) return set_error(PPE_NOT_CONVERGED, "tridiagonal QR did not converge");
  eigvecs_host(n, a, sw, Z);
  const std::vector<int> ord = ascending(a);
  for (int j = 0; j < n; ++j) theta[j] = a[ord[j]];
  if (U) std::copy(Z.begin(), Z.end(), U);
  return PPE_OK;
}

extern "C" void ppe_ritz_destroy(ppe_ritz* r) {
  if (!r) return;
  dev_free(r->d_V);
  dev_free(r->d_U);
  delete r;
}

#define HIPCHK_R(call)                                                               \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) {                                                          \
      cleanup();                                                                     \
      ppe_ritz_destroy(r);                                                           \
      return set_error(PPE_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    }                                                                                \
  } while (0)

extern "C" ppe_status ppe_ritz_create(ppe_problem* p, int32_t m, const double* v0, ppe_ritz** out, hipStream_t s) {
  if (!p || !v0 || !out) return set_error(PPE_ERR_INVALID_ARG, "problem, v0 or out is NULL");
  *out = nullptr;
  if (p->mask_mode == PPE_MASK_SOLID) return reject_solid(p, "ppe_ritz_create");
  const int64_t N = (int64_t)p->nx * p->ny;
  if (m < 1 || m > 8192 || m >= N) return set_error(PPE_ERR_INVALID_ARG, "m must lie in [1, min(8192, N - 1)]");
  ppe_ritz* r = new ppe_ritz();
  r->nx = p->nx;
  r->ny = p->ny;
  r->N = N;
  r->d_V = (double*)dev_alloc(sizeof(double) * (size_t)(m + 1) * N);
  double* d_w = (double*)dev_alloc(sizeof(double) * N);
  double* d_c = (double*)dev_alloc(sizeof(double) * (m + 1));
  double* d_ab = (double*)dev_alloc(sizeof(double) * 2 * m);  // alpha [m], beta [m]
  double* d_part = (double*)dev_alloc(sizeof(double) * kNormBlocks);
  auto cleanup = [&]() {
    dev_free(d_w);
    dev_free(d_c);
    dev_free(d_ab);
    dev_free(d_part);
    d_w = d_c = d_ab = d_part = nullptr;
  };
  if (!r->d_V || !d_w || !d_c || !d_ab || !d_part) {
    cleanup();
    ppe_ritz_destroy(r);
    return set_error(PPE_ERR_HIP, "allocation of the Lanczos basis (%d x %lld) failed", m + 1, (long long)N);
  }
  double* V = r->d_V;
  const unsigned gN = blocks_for(N);
  k_fill<<<gN, kRB, 0, s>>>(V, N, 1.0 / std::sqrt((double)N));
  k_fill<<<blocks_for(2 * m), kRB, 0, s>>>(d_ab, 2 * m, 0.0);
  // v_0: the start vector without its mean, normalised. Its norm before and
  // after the projection tells a zero or constant start vector.
  HIPCHK_R(hipMemcpyAsync(d_w, v0, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
  std::vector<double> part_in(kNormBlocks);
  k_sumsq64<<<kNormBlocks, kRB, 0, s>>>(d_w, N, d_part);
  HIPCHK_R(hipMemcpyAsync(part_in.data(), d_part, sizeof(double) * kNormBlocks, hipMemcpyDeviceToHost, s));
  for (int pass = 0; pass < 2; ++pass) {
    k_rows_dot<<<1, kRB, 0, s>>>(V, N, d_w, d_c);
    k_rows_sub<<<gN, kRB, 0, s>>>(V, 1, N, d_c, d_w, 0, d_ab + m);  // scratch accumulator, cleared below
  }
  k_sumsq64<<<kNormBlocks, kRB, 0, s>>>(d_w, N, d_part);
  k_next_vector<<<gN, kRB, 0, s>>>(d_w, N, d_part, 0.0, V + N, d_ab + m);
  HIPCHK_R(hipGetLastError());
  double nrm0 = 0.0;  // the projected norm, in beta[0] for now
  HIPCHK_R(hipMemcpyAsync(&nrm0, d_ab + m, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK_R(hipStreamSynchronize(s));
  double nrm_in = 0.0;
  for (double v : part_in) nrm_in += v;
  nrm_in = std::sqrt(nrm_in);
  if (!std::isfinite(nrm_in) || !std::isfinite(nrm0) || !(nrm0 > 1e-10 * nrm_in)) {
    cleanup();
    ppe_ritz_destroy(r);
    return set_error(PPE_ERR_INVALID_ARG, "start vector is zero, constant or non-finite");
  }
  k_fill<<<blocks_for(m), kRB, 0, s>>>(d_ab + m, m, 0.0);
  // Lanczos steps. An exhausted Krylov space shows as a beta at rounding level;
  // the host truncates there after the run (later rows are then unused).
  for (int j = 0; j < m; ++j) {
    double* vj = V + (size_t)(j + 1) * N;
    launch_apply_f64(p->coef, 1, vj, d_w, 4, s);
    for (int pass = 0; pass < 2; ++pass) {
      k_rows_dot<<<j + 2, kRB, 0, s>>>(V, N, d_w, d_c);
      k_rows_sub<<<gN, kRB, 0, s>>>(V, j + 2, N, d_c, d_w, j + 1, d_ab + j);
    }
    if (j + 1 < m) {
      k_sumsq64<<<kNormBlocks, kRB, 0, s>>>(d_w, N, d_part);
      k_next_vector<<<gN, kRB, 0, s>>>(d_w, N, d_part, 0.0, V + (size_t)(j + 2) * N, d_ab + m + j);
    }
  }
  HIPCHK_R(hipGetLastError());
  std::vector<double> ab(2 * m);
  HIPCHK_R(hipMemcpyAsync(ab.data(), d_ab, sizeof(double) * 2 * m, hipMemcpyDeviceToHost, s));
  HIPCHK_R(hipStreamSynchronize(s));
  cleanup();
  // Truncate at the first exhausted step.
  double amax = 0.0;
  for (int j = 0; j < m; ++j) amax = std::max(amax, std::fabs(ab[j]));
  int mk = m;
  for (int j = 0; j + 1 < m; ++j)
    if (!(ab[m + j] > 1e-12 * amax)) {
      mk = j + 1;
      break;
    }
  for (int j = 0; j < m; ++j)
    if (!std::isfinite(ab[j]) || !std::isfinite(ab[m + j])) {
      ppe_ritz_destroy(r);
      return set_error(PPE_ERR_NONFINITE, "non-finite Lanczos coefficient at step %d", j);
    }
  r->m = mk;
  r->alpha.assign(ab.begin(), ab.begin() + mk);
  r->beta.assign(ab.begin() + m, ab.begin() + m + (mk - 1));
  std::vector<double> a = r->alpha, b = r->beta;
  QrSweeps sw;
  if (!tridiag_qr(mk, a, b, sw)) {
    ppe_ritz_destroy(r);
    return set_error(PPE_NOT_CONVERGED, "tridiagonal QR did not converge");
  }
  const std::vector<int> ord = ascending(a);
  r->theta.resize(mk);
  for (int j = 0; j < mk; ++j) r->theta[j] = a[ord[j]];
  r->d_U = (double*)dev_alloc(sizeof(double) * (size_t)mk * mk);
  if (!r->d_U) {
    ppe_ritz_destroy(r);
    return set_error(PPE_ERR_HIP, "allocation of the Ritz eigenvectors failed");
  }
  const ppe_status est = eigvecs_device(mk, a, sw, r->d_U, s);
  if (est != PPE_OK) {
    ppe_ritz_destroy(r);
    return est;
  }
  *out = r;
  return PPE_OK;
}

extern "C" ppe_status ppe_ritz_info(const ppe_ritz* r, int32_t* m, double* alpha, double* beta, double* theta) {
  if (!r) return set_error(PPE_ERR_INVALID_ARG, "ritz is NULL");
  if (m) *m = r->m;
  if (alpha) std::copy(r->alpha.begin(), r->alpha.end(), alpha);
  if (beta) std::copy(r->beta.begin(), r->beta.end(), beta);
  if (theta) std::copy(r->theta.begin(), r->theta.end(), theta);
  return PPE_OK;
}

extern "C" ppe_status ppe_ritz_rhs(const ppe_ritz* r, int32_t nb, uint64_t seed, int64_t step, double b,
                                   double scale, float* R, hipStream_t s) {
  if (!r || !R) return set_error(PPE_ERR_INVALID_ARG, "ritz or R is NULL");
  if (!(scale > 0.0) || !std::isfinite(scale)) return set_error(PPE_ERR_INVALID_ARG, "scale must be finite and > 0");
  if (nb < 1 || nb > 4096) return set_error(PPE_ERR_INVALID_ARG, "nb must lie in [1, 4096]");
  if (!(b >= 0.0 && b <= 1.0)) return set_error(PPE_ERR_INVALID_ARG, "b must lie in [0, 1]");
  const int m = r->m;
  const int64_t N = r->N;
  double* d_c = (double*)dev_alloc(sizeof(double) * (size_t)m * nb);
  double* d_y = (double*)dev_alloc(sizeof(double) * (size_t)m * nb);
  double* d_r = (double*)dev_alloc(sizeof(double) * (size_t)N * nb);
  double* d_part = (double*)dev_alloc(sizeof(double) * kNormBlocks * nb);
  auto cleanup = [&]() {
    dev_free(d_c);
    dev_free(d_y);
    dev_free(d_r);
    dev_free(d_part);
  };
  if (!d_c || !d_y || !d_r || !d_part) {
    cleanup();
    return set_error(PPE_ERR_HIP, "allocation of the Ritz batch buffers failed");
  }
  const int jmax = (int)std::floor(b * m);
  k_ritz_coef<<<blocks_for((int64_t)m * nb), kRB, 0, s>>>(m, nb, jmax, (uint32_t)seed, (uint32_t)(seed >> 32),
                                                         (uint32_t)(uint64_t)step, (uint32_t)((uint64_t)step >> 32),
                                                         d_c);
  k_u_times_c<<<dim3(m, nb), kRB, 0, s>>>(r->d_U, m, d_c, d_y);
  k_v_times_y<<<dim3(blocks_for(N), nb), kRB, 0, s>>>(r->d_V, m, N, d_y, d_r);
  k_sumsq64_batch<<<dim3(kNormBlocks, nb), kRB, 0, s>>>(d_r, N, d_part);
  k_normalise<<<dim3(kNormBlocks, nb), kRB, 0, s>>>(d_r, N, d_part, scale, R);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  cleanup();
  if (e != hipSuccess) return set_error(PPE_ERR_HIP, "Ritz batch: %s", hipGetErrorString(e));
  return PPE_OK;
}
