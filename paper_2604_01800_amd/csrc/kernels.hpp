// Host-side declarations of the kernel launchers.
#pragma once
#include "common.hpp"

namespace ppe {

// Arguments of the PCG kernels (passed by value; pointers are device memory).
struct PcgArgs {
  Coef c;
  int P;             // workgroups per solve
  int R;             // rows per wavefront
  int64_t N;         // cells per solve
  float *xc, *r, *p0, *p1;  // [nb][N] each
  float* r1;                // [nb][N] second residual buffer (single-reduction iteration)
  double *partA, *partB;    // [nb][P], [nb][2][P]
  double* part1;            // [2][nb][5][P] sums of the single-reduction iteration
  int P2;                   // workgroups per solve of the two-iteration form (56-column tiles)
  double* part2;            // [2][nb][11][P2] sums of the two-iteration form
  double* partD;            // [nb][3][P] line-search partial sums
  const float* e;           // [nb][N] line-search direction
  SolveState* st;           // [nb]
  int32_t* flags;           // [nb] done codes
  const CallArgs* call;
  double tol;
  int tol_kind;
  int jacobi;
  int zero_x0;  // the setup zeroes x before the first residual
  // Multigrid preconditioner (host-side handle, NULL otherwise): the two-phase
  // kernels then read z = M^-1 r from z, which the V-cycle writes after every
  // pass that changes r.
  const struct MgData* mg;
  float* z;     // [nb][N]
  // Incomplete-Cholesky preconditioner (red-black IC(0)): 1/D on red cells
  // and 1/S on black cells [ny][nx], NULL otherwise; z as for multigrid.
  const float* icq;
  // Residual history (device [nb][hist_cap] FP64, NULL when not recorded).
  double* hist;
  int hist_cap;
};

dim3 stencil_grid(const Coef& c, int R, int nb);
dim3 stencil_grid2(const Coef& c, int R, int nb);
void launch_apply_f32(const Coef& c, int nb, const float* x, float* y, int R, hipStream_t s);
void launch_apply_f64(const Coef& c, int nb, const double* x, double* y, int R, hipStream_t s);
void launch_rhs_to_source(const Coef& c, int nb, const float* b, float* f, hipStream_t s);
void launch_ic(const PcgArgs& a, int nb, hipStream_t s);
void launch_set_call(CallArgs* c, const float* f, double* x, int max_iter, double delta2, hipStream_t s);
void launch_rhs(const PcgArgs& a, int nb, hipStream_t s);
void launch_pcg_setup(const PcgArgs& a, int nb, hipStream_t s);
void launch_pcg1_setup(const PcgArgs& a, int nb, hipStream_t s);
void launch_pcg1_step(const PcgArgs& a, int nb, int par, hipStream_t s);
void launch_pcg1_init(const PcgArgs& a, int nb, hipStream_t s);
void launch_pcg1_multi_step(const PcgArgs* descs, const uint32_t* work, int nblocks, int R, bool jacobi, int par,
                            hipStream_t s);
void launch_pcg1_step_timed(const PcgArgs& a, int nb, int par, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
void launch_pcg2_setup(const PcgArgs& a, int nb, hipStream_t s);
void launch_pcg2_step(const PcgArgs& a, int nb, int par, hipStream_t s);
void launch_pcg2_multi_step(const PcgArgs* descs, const uint32_t* work, int nblocks, int R, bool jacobi, int par,
                            hipStream_t s);
void launch_pcg2_step_timed(const PcgArgs& a, int nb, int par, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
void launch_pcg_pair(const PcgArgs& a, int nb, int par, int force, int force_restart, hipStream_t s);
void launch_pcg_phase_a(const PcgArgs& a, int nb, int par, hipStream_t s);
void launch_pcg_phase_b(const PcgArgs& a, int nb, int par, hipStream_t s);
void launch_copy16(const void* src, void* dst, int64_t n16, hipStream_t s);
void launch_pcg_phase_timed(const PcgArgs& a, int nb, int par, int phase, hipStream_t s, hipEvent_t e0,
                            hipEvent_t e1);
void launch_direction(const PcgArgs& a, int nb, int mode, float* e, hipStream_t s);
void launch_dlsm_step(const PcgArgs& a, int nb, int par, hipStream_t s);
// Hybrid phase clock: time since the last mark is added to phase cat
// (0 CG-type, 1 network, 2 line search; -1 marks only).
void launch_mark(const PcgArgs& a, int nb, int cat, hipStream_t s);
void launch_zero_flags(int32_t* flags, int nb, hipStream_t s);
// Residual-history entry after a CG block (no-op without a history buffer).
void launch_hist_cg(const PcgArgs& a, int nb, int par, hipStream_t s);
void launch_apply_multi(const Coef* coefs, int nx, int ny, int nb, const float* x, float* y, hipStream_t s);
void launch_pcg_finish(const PcgArgs& a, int nb, hipStream_t s);
// The multigrid V-cycle on the residual a.r into a.z (a.mg), ending with the
// partial sums of r.z in the second half of a.partB.
void launch_vcycle(const PcgArgs& a, int nb, hipStream_t s);

}  // namespace ppe
