// Shared device-side definitions of the MI355X PPE library (HIP, gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ppe {

constexpr int kWave = 64;    // CDNA wavefront width
constexpr int kWaves = 4;    // wavefronts per stencil workgroup
constexpr int kBlock = kWave * kWaves;

// 1D coefficient arrays of one tensor grid (device memory). The operator of
// Eq. 10 in finite-volume form needs only these O(nx + ny) numbers:
//   (A v)_ij = hy_j [gx_{i+1}(v_ij - v_{i+1,j}) + gx_i (v_ij - v_{i-1,j})]
//            + hx_i [gy_{j+1}(v_ij - v_{i,j+1}) + gy_j (v_ij - v_{i,j-1})]
// gx[k] = 1/(xc[k] - xc[k-1]) for the interior x-face k, 0 at the walls.
// The arrays are zero-padded in memory: indices in [-kPadX, n + kPadX) for
// hx/gx and [-kPadY0, n + kPadY1) for hy/gy are valid and read 0 off the grid.
constexpr int kPadX = 128, kPadY0 = 32, kPadY1 = 128;
struct Coef {
  int nx, ny;
  const float *hx, *hy, *gx, *gy;          // [nx], [ny], [nx+1], [ny+1]
  const double *hx64, *hy64, *gx64, *gy64; // same in FP64
  const double *xc64, *yc64;               // cell centres [nx], [ny] (not padded)
  // Solid-mask operator (NULL otherwise): only faces between two fluid cells
  // carry weight and solid cells have identity rows. fl is the fluid
  // indicator (1 fluid, 0 solid), dinv the inverse of that operator's
  // diagonal (1 on solid cells), both [ny][nx]; nfluid counts the fluid cells.
  const float* fl;
  const float* dinv;
  int64_t nfluid;
};

// Per-solve iteration state. Fields with a [2] index are written by the
// kernel of that parity and read by the next kernels, so no workgroup reads a
// slot that another workgroup of the same launch writes.
struct SolveState {
  double rho[2];      // r.z of the current residual (phase A)
  double alpha[2];    // CG step length (phase B); 0 after a true-residual pass
  double rr_ru[2];    // ||r_true||^2 at the last reliable update (phase A)
  double rr_last[2];  // last recursive ||r||^2 seen by phase A
  int32_t it[2];      // iterations completed (CG + line search)
  int32_t n_ru[2];    // reliable updates done
  int32_t mode[2];    // what phase B of this parity does: 0 CG update, 1 true residual
  int32_t restart[2]; // next CG step uses beta = 0
  int32_t brk[2];     // phase B hit p.Ap <= 0 (breakdown)
  int32_t it_cg[2];
  int32_t dflag[2];   // done code as seen after phase A of this parity
  // written once per solve
  double bmean, bnorm2, thr2, xmean;
  double rr_final;
  int32_t nonfinite;
  int32_t done;       // 0 running, 1 converged, 2 iteration limit, 3 non-finite
  int32_t it_final, nru_final, itcg_final;
  // line-search step (hybrid): counters and the hand-over between its two kernels
  int32_t n_dlsm, n_rej;
  int32_t dl_active, dl_it;
  double dl_alpha;
  int32_t pad[2];
  // device real-time clock (wall_clock64) at set-up and when the solve finished
  uint64_t t_start, t_done;
  // hybrid solve: clock at the last phase mark and the time accumulated per
  // phase (0 CG-type iterations, 1 network forwards, 2 line-search kernels)
  uint64_t t_mark;
  uint64_t t_acc[3];
};

// MODE_FLUSH and MODE_SUMS are used by the single-reduction iteration only
// (x += x_c, then MODE_TRUE, then MODE_SUMS before the next CG step).
enum : int32_t { MODE_CG = 0, MODE_TRUE = 1, MODE_FLUSH = 2, MODE_SUMS = 3 };
enum : int32_t { DONE_NO = 0, DONE_CONV = 1, DONE_MAXIT = 2, DONE_NONFINITE = 3 };

// Per-call pointers kept in device memory so that a captured graph can be
// replayed for new caller buffers.
struct CallArgs {
  const float* f;  // [nb][ny][nx]
  double* x;       // [nb][ny][nx]
  int32_t max_iter;
  int32_t pad;
  double delta2;   // reliable-update trigger (delta^2)
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Sum over a 256-thread workgroup; every thread gets the same bits.
__device__ __forceinline__ double block_sum(double v, double* lds) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) lds[threadIdx.x / kWave] = v;
  __syncthreads();
  return ((lds[0] + lds[1]) + lds[2]) + lds[3];
}

// Fixed-order sum of P per-workgroup partials; identical in every workgroup.
__device__ __forceinline__ double reduce_partials(const double* part, int P, double* lds) {
  double s = 0.0;
  for (int k = threadIdx.x; k < P; k += kBlock) s += part[k];
  return block_sum(s, lds);
}

__device__ __forceinline__ bool is_first_block() {
  return blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0;
}

}  // namespace ppe
