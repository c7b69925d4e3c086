/*
 * ppe.h — C-ABI of the MI355X pressure-Poisson library.
 *
 * The library solves the pressure Poisson equation of the fractional-step
 * method (Eq. 7, recast as M dp = S in Eq. 10) on a tensor-product stretched
 * Cartesian grid, either with (Jacobi-)preconditioned conjugate gradients or in
 * the hybrid form of Sec. 2.2, where a DeepONet with a grid-spacing-aware U-Net
 * branch (Sec. 2.4) supplies line-search directions (Eqs. 11-13) between blocks
 * of CG iterations. The network is trained by the library on fabricated
 * systems with the residual loss of Eq. 19.
 *
 * Discretisation (the reading of M used throughout): cell-centred finite
 * volumes, each interior face weighted by (face length)/(centre distance),
 * boundary faces dropped (homogeneous Neumann). For the PDE -lap p = f the
 * library builds b = (cell area) * f and removes the plain mean of b
 * (compatibility with the constant null space). The returned x is the
 * minimum-norm solution (zero plain mean). The time step of Eq. 7 is absorbed
 * into f.
 *
 * Conventions
 *   - Arrays on a grid are row-major [ny][nx], index j*nx + i, and batches are
 *     [nb][ny][nx]. "device" pointers are HIP device memory on the current
 *     device, "host" pointers are ordinary host memory.
 *   - The caller owns every data pointer. *_create copies the host grid arrays;
 *     the library never keeps caller pointers beyond a call.
 *   - Work is enqueued on the given stream (0 = the default stream). Solve and
 *     train calls return after the stream's work for the call has completed,
 *     since convergence is polled and statistics are host values.
 *   - Handles are not thread-safe: use one handle per thread.
 *   - Every entry point validates its arguments before launching anything and
 *     returns a status; ppe_last_error() gives a thread-local message.
 */
#ifndef PPE_H
#define PPE_H

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ppe_status;
enum {
  PPE_OK = 0,
  PPE_NOT_CONVERGED = 1,   /* x = best iterate (after a final true-residual update), stats valid */
  PPE_ERR_INVALID_ARG = -1,
  PPE_ERR_SHAPE = -2,      /* nx, ny not divisible by 2^(levels-1), or net/grid mismatch */
  PPE_ERR_UNSUPPORTED = -3,
  PPE_ERR_HIP = -4,        /* a HIP runtime call failed; see ppe_last_error() */
  PPE_ERR_NONFINITE = -5   /* NaN/Inf in the source f, or produced by the iteration */
};

typedef struct ppe_problem ppe_problem; /* opaque: one grid, its coefficients and workspaces */
typedef struct ppe_net ppe_net;         /* opaque: DeepONet weights, optimiser state, buffers */

/* CG-type of the solve (Sec. 2.5): vanilla CG, Jacobi-PCG, multigrid-
 * preconditioned CG (the paper's MGPCG-4): a V-cycle on the tensor grid with
 * levels made by merging 2 x 2 cells, Galerkin coarse operators of the
 * piecewise-constant prolongation, a degree-2 Chebyshev smoother on D^-1 A
 * over [0.2, 2] before and after the coarse correction, and an exact
 * separable solve on the coarsest level (opts->mg_levels levels, default 4);
 * or incomplete-Cholesky PCG (the paper's ICPCG): IC(0) of the operator in
 * red-black (checkerboard) ordering, whose two triangular solves are two
 * passes over independent cells (nx and ny at least 2, else PPE_ERR_SHAPE). */
enum { PPE_PC_NONE = 0, PPE_PC_JACOBI = 1, PPE_PC_MG = 2, PPE_PC_IC = 3 };
enum { PPE_TOL_RELATIVE = 0, PPE_TOL_ABSOLUTE = 1 };   /* ||b-Ax||2 <= tol*||b||2 or <= tol */

/* How an obstacle mask enters the operator. DIBPM (default): it does not;
 * the decoupled immersed-boundary projection method keeps the coefficient
 * matrix of the PPE unchanged by the body (Sec. 2.1, Eqs. 4-5; the forcing
 * acts through the source), and the mask is an input channel of the network.
 * SOLID: faces between a fluid and a solid cell are removed and solid cells
 * get identity rows (x = b there), the classical masked Laplacian; it is not
 * the paper's form and is offered for comparison (ppe_apply_*, and the plain
 * solve with the two-phase iteration and no or Jacobi preconditioning;
 * other solves return PPE_ERR_UNSUPPORTED). */
enum { PPE_MASK_DIBPM = 0, PPE_MASK_SOLID = 1 };

/* Form of the plain PCG iteration (the same iterates in exact arithmetic):
 * SINGLE_REDUCTION regroups the recurrences so that one launch and one
 * grid-wide reduction make an iteration (p.Ap from an exact expansion in
 * sums of the previous launch); TWO_PHASE is the textbook order with two
 * reductions per iteration; TWO_STEP makes two iterations per launch and
 * per reduction (s-step CG with s = 2: the second iteration's scalars are
 * exact expansions in eleven sums of the previous launch, and every
 * workgroup carries a 4-cell halo). A launch of TWO_STEP may do a single
 * iteration (next to max_iter, or when the expansion is not positive), so
 * iteration counts keep their meaning. AUTO takes the problem's tuned
 * choice for the batch size (ppe_tune_pcg, ppe_set_tuning), else TWO_STEP
 * (the fastest form on MI355X at every size measured, 256^2 to 2 x 2048^2). The
 * hybrid solve always uses TWO_PHASE; the mixed-size batch (ppe_solve_batch)
 * runs TWO_STEP for AUTO and TWO_STEP, SINGLE_REDUCTION on request, and
 * rejects TWO_PHASE. */
enum { PPE_PCG_AUTO = 0, PPE_PCG_SINGLE_REDUCTION = 1, PPE_PCG_TWO_PHASE = 2, PPE_PCG_TWO_STEP = 3 };

/* Error-direction provider of the hybrid solve. NET is the DeepONet; the others
 * replace it for testing the controller and its fallback. */
enum {
  PPE_DIR_NET = 0,
  PPE_DIR_ZERO = 1,    /* e = 0: every line-search step is rejected */
  PPE_DIR_JACOBI = 2,  /* e = D^-1 r */
  PPE_DIR_NAN = 3,     /* e = NaN: every step is rejected */
  PPE_DIR_ONES = 4     /* e = 1 (null space, e^T A e = 0): rejected */
};

/* Grid description (Sec. 2.5 / Table 1: a stretched Cartesian grid).
 * xc, yc: host, [nx], [ny] strictly increasing cell centres.
 * hx, hy: host, [nx], [ny] cell widths > 0 (face length of the other axis).
 * At most 2^28 cells (16384^2) per grid.
 * mask:   host [ny*nx] or NULL, 1 = solid; an input channel of the network.
 * mask_mode: PPE_MASK_DIBPM (0, the mask does not enter M) or
 *         PPE_MASK_SOLID (needs a mask with at least one fluid cell). */
typedef struct {
  int32_t nx, ny;
  const double *xc, *yc;
  const double *hx, *hy;
  const uint8_t* mask;
  int32_t mask_mode;
} ppe_grid_desc;

typedef struct {
  double tol;              /* default 1e-6 */
  int32_t tol_kind;        /* PPE_TOL_RELATIVE (default) or PPE_TOL_ABSOLUTE */
  int32_t precond;         /* PPE_PC_JACOBI (default) or PPE_PC_NONE */
  int32_t max_iter;        /* iterations (CG + line search) before giving up */
  int32_t num_cg;          /* hybrid: CG iterations per round (default 3) */
  int32_t num_dlsm;        /* hybrid: line-search steps per round (default 2) */
  int32_t direction;       /* hybrid: PPE_DIR_* (default PPE_DIR_NET) */
  double reliable_delta;   /* true-residual update when ||r|| < delta*||r_true|| (default 0.3) */
  int32_t rows_per_wave;   /* stencil tile height per wavefront: 0 = tuned or default, else 2,4,8,16
                              (the two-step form also 20, 24) */
  int32_t use_graph;       /* 1 (default) = replay iteration chunks as a HIP graph, 0 = eager launches */
  int32_t chunk;           /* iterations per polled chunk (0 = default 64) */
  int32_t zero_x0;         /* 1 = ignore x on entry and start from x0 = 0 */
  int32_t variant;         /* plain solve: PPE_PCG_AUTO (default), _SINGLE_REDUCTION, _TWO_PHASE or _TWO_STEP;
                              PPE_PC_MG, PPE_PC_IC, PPE_MASK_SOLID and record_history run the
                              two-phase form */
  int32_t mg_levels;       /* PPE_PC_MG: levels of the V-cycle, 0 = default 4, at most 12; nx and ny must
                              be divisible by 2^(levels-1) (else PPE_ERR_SHAPE) */
  int32_t record_history;  /* 1 = fill each solve's stats history (the caller's buffer, see below) */
} ppe_solve_opts;

typedef struct {
  int32_t status;          /* per solve: PPE_OK / PPE_NOT_CONVERGED / PPE_ERR_NONFINITE */
  int32_t iters_total, iters_cg, iters_dlsm, dlsm_rejected, reliable_updates;
  double rel_res_true;     /* FP64 ||b - A x||2 / ||b||2 at exit */
  double abs_res_true;     /* FP64 ||b - A x||2 at exit */
  double bnorm;            /* ||b||2 after projection */
  double rhs_mean_removed; /* plain mean removed from b = area * f */
  double ms_total;         /* wall time of the call (host clock), same for all solves of a call */
  double ms_device;        /* this solve's time from its set-up to its convergence decision, on the
                              device's real-time clock (per solve within a batch) */
  /* Split of the hybrid solve's device time (Tables 2-3 report the DLSM share):
   * ms_pcg the CG-type iterations (with their reliable updates and
   * preconditioner), ms_net the network forwards, ms_dlsm the line-search
   * vector kernels; device real-time clock, summed over the replayed rounds
   * (per call, shared by the solves of a batch). Plain solves: ms_pcg =
   * ms_device, the others 0. */
  double ms_pcg, ms_net, ms_dlsm;
  /* Residual history, with opts->record_history: the caller sets history (a
   * host buffer of history_cap doubles, or NULL) and history_cap before the
   * call; the library fills history[k] = ||r_k||_2 / ||b||_2 (the recursive
   * residual after iteration k, CG or line search; k = 0 the start, and at a
   * reliable update the true residual) for k < min(history_cap, iters + 1),
   * and sets history_len to that count. Every other field is output only. */
  double* history;
  int32_t history_cap, history_len;
} ppe_solve_stats;

/* Network configuration (Sec. 2.4). Defaults (ppe_net_config_default): 4 levels,
 * 32 base channels doubling per level, inputs (scaled residual, mask), 128-term
 * DeepONet basis, trunk 2 -> 128 x 4 -> 128 (tanh), per-layer weight network
 * 4 -> 16 (tanh) -> 1 for the Mesh-Conv local weight of each node (Eq. 17).
 * Limits: levels in [2, 6]; base_channels a multiple of 8 with
 * base_channels x 2^(levels-1) <= 1024 (the paper's U-Net, 5 levels from 40
 * channels, fits); basis and trunk_width multiples of 8 in [8, 128];
 * trunk_hidden in [1, 8]; phi_hidden in [1, 32]. Other values give
 * PPE_ERR_INVALID_ARG. Training (ppe_net_train_step) further needs every
 * Mesh-Conv layer's inputs x phi_hidden to fit the local-weight backward's
 * LDS (up to about 850 inputs at phi_hidden 16, 200 at phi_hidden 32), else
 * PPE_ERR_INVALID_ARG. */
typedef struct {
  int32_t levels, base_channels, basis, trunk_width, trunk_hidden, phi_hidden;
  int32_t use_eta;         /* Mesh-Conv local weight (Eqs. 17-18): 2 = one weight per node multiplying the
                              whole feature vector, as the equations are written (default); 1 = one
                              weight per input channel (Phi with C_in outputs); 0 = standard conv
                              (the "-Conv" ablation) */
  int32_t use_spacing;     /* 1 = concatenate the normalised widths (hx, hy) at each level */
} ppe_net_config;

typedef struct {
  float lr, beta1, beta2, eps;  /* Adam; defaults 1e-3, 0.9, 0.999, 1e-8 */
  uint64_t seed;                /* data generator seed (used when R == NULL) */
  int64_t step;                 /* data generator step counter (>= 0) */
  /* Data generator (ppe_generate_rhs, and ppe_net_train_step with R == NULL):
   * Gaussian random fields with squared-exponential covariance of length
   * scale l, log-uniform in [grf_len_lo, grf_len_hi] per sample (defaults
   * 0.05, 0.5; FP32 values), from grf_features random Fourier features
   * (default 512). */
  float grf_len_lo, grf_len_hi;
  int32_t grf_features;
  float clip_norm;              /* > 0: scale the gradient to this L2 norm before Adam when larger (default 0) */
  float sam_rho;                /* > 0: sharpness-aware step (Sec. 2.4): the gradient Adam uses is taken at
                                   w + sam_rho g / |g| (two forward/backward passes; default 0) */
  int32_t loss_kind;            /* PPE_LOSS_RESIDUAL (default, Eq. 19), PPE_LOSS_SUPERVISED or PPE_LOSS_ANORM */
} ppe_train_opts;

/* Training loss. RESIDUAL is Eq. 19, mean over cells of (R - A NN(R))^2.
 * SUPERVISED compares the network output with a target error field e*
 * (typically the FP64 solution of A e* = R): since the line search of
 * Eqs. 12-13 is blind to the output's scale and to constants (A 1 = 0), the
 * loss is scale- and shift-invariant: with y0 = y - mean(y),
 * L = 1 - (y0 . e*)^2 / (|y0|^2 |e*|^2) per sample (0 when y0 is a multiple of
 * e*), averaged over the batch.
 * ANORM is one minus the share of the A-norm error that one exact line
 * search along the output removes (the DLSM step of Eqs. 12-13 with e* the
 * error): L = 1 - (R . y)^2 / ((y . A y)(R . e*)) per sample, averaged over
 * the batch; scale- and shift-invariant like SUPERVISED, but the misfit is
 * weighted by A once (Eq. 19 weights it by A^2, SUPERVISED not at all). A
 * sample with y . A y <= 0 or R . e* <= 0 counts 1 with no gradient. Both
 * SUPERVISED and ANORM are options beside the paper's Eq. 19. */
enum { PPE_LOSS_RESIDUAL = 0, PPE_LOSS_SUPERVISED = 1, PPE_LOSS_ANORM = 2 };

/* ---- problem: per-grid setup, built once and reused. The coefficient
 *      matrix of the PPE stays constant over a simulation, so its
 *      preconditioner is built at the first time step and reused in all
 *      later ones (Sec. 2.5, technical details); a problem handle holds the
 *      grid's operator coefficients and workspaces in the same way. ---- */
/* Copies the grid to the device with copies ordered on stream s (then
 * synchronises s). */
ppe_status ppe_problem_create(const ppe_grid_desc* grid, hipStream_t s, ppe_problem** out);
void ppe_problem_destroy(ppe_problem* p);
void ppe_solve_opts_default(ppe_solve_opts* o);

/* y = A x, the operator of Eq. 10 (FP32 or FP64 arithmetic).
 * x, y: device [nb][ny][nx]. */
ppe_status ppe_apply_f32(const ppe_problem* p, int32_t nb, const float* x, float* y, hipStream_t s);
ppe_status ppe_apply_f64(const ppe_problem* p, int32_t nb, const double* x, double* y, hipStream_t s);

/* f = b / (cell area), elementwise in FP64 rounded to FP32: the source
 * whose right-hand side (Eq. 10, b = cell area x f) is b, so that a caller
 * holding right-hand sides (the training vectors of Eqs. 15-16, for one)
 * can solve A x = b with ppe_solve_plain. b, f: device FP32 [nb][ny][nx];
 * may alias. Enqueued on s; does not synchronise. */
ppe_status ppe_rhs_to_source(const ppe_problem* p, int32_t nb, const float* b, float* f, hipStream_t s);

/* z = M^-1 r for the preconditioner opts->precond selects (opts NULL:
 * defaults): PPE_PC_JACOBI z = D^-1 r; PPE_PC_MG one V-cycle from a zero
 * guess (opts->mg_levels), the operator the MG-PCG solve applies each
 * iteration; PPE_PC_IC the two triangular solves of red-black IC(0);
 * PPE_PC_NONE z = r. r, z: device FP32 [nb][ny][nx]. Returns
 * after the stream's work for the call has completed. */
ppe_status ppe_apply_precond(ppe_problem* p, int32_t nb, const float* r, float* z, const ppe_solve_opts* opts,
                             hipStream_t s);

/* Plain (Jacobi-)PCG solve of nb systems on one grid (Sec. 2.5, JPCG).
 * f: device FP32 [nb][ny][nx], the source of -lap p = f (pointwise values).
 * x: device FP64 [nb][ny][nx]; in: initial guess, out: solution with zero mean.
 * stats: host [nb] or NULL. Vectors are FP32; dot products, the solution
 * accumulator and the convergence judge (true residual) are FP64.
 * Returns PPE_OK if every solve converged, PPE_NOT_CONVERGED if any did not,
 * PPE_ERR_NONFINITE if any source held NaN/Inf. */
ppe_status ppe_solve_plain(ppe_problem* p, int32_t nb, const float* f, double* x,
                           const ppe_solve_opts* opts, ppe_solve_stats* stats, hipStream_t s);

/* Plain (Jacobi-)PCG solves of n systems on grids of different sizes, one
 * right-hand side per grid, batched into one launch per two iterations
 * (two-step form) or per iteration (single-reduction form, on request via
 * opts->variant): a work list of (solve, workgroup) entries over all grids.
 * Each solve's result is bit-identical to the same solve alone with the same
 * form and tile height.
 * problems: host array of n distinct problems; f: host array of n device
 * FP32 sources [ny_i][nx_i]; x: host array of n device FP64 solutions
 * (in: initial guess, out: zero-mean solution); stats: host [n] or NULL,
 * with ms_device the solve's own time to its convergence decision.
 * net: NULL for the plain solves above. Otherwise each system gets the hybrid
 * solve of ppe_solve_hybrid (Sec. 2.2, with opts->direction, num_cg and
 * num_dlsm checked as there; the network must fit every grid when the
 * direction is PPE_DIR_NET). The solves' rounds advance in lock step on
 * stream s, and each solve is bit-identical to the same ppe_solve_hybrid
 * call alone. With PPE_DIR_NET every line-search step runs the network on
 * all undecided solves as one grouped launch per layer (the forward of
 * ppe_net_forward_batch), and the phase times of each solve (ms_pcg, ms_net,
 * ms_dlsm) are those of the whole lock-step batch; other directions replay
 * each undecided solve's round in turn. The network is only read. Statuses
 * as for ppe_solve_plain. */
ppe_status ppe_solve_batch(int32_t n, ppe_problem* const* problems, const ppe_net* net, const float* const* f,
                           double* const* x, const ppe_solve_opts* opts, ppe_solve_stats* stats, hipStream_t s);

/* Hybrid solve (Sec. 2.2): rounds of num_cg PCG iterations and num_dlsm
 * line-search steps along e = NN(r) (Eqs. 12-13), restarting PCG after each
 * line-search block; convergence judged on the FP64 true residual. net may be
 * NULL when opts->direction != PPE_DIR_NET. Same arrays as ppe_solve_plain.
 * Requires nx, ny divisible by 2^(levels-1) when the network is used. */
ppe_status ppe_solve_hybrid(ppe_problem* p, ppe_net* net, int32_t nb, const float* f, double* x,
                            const ppe_solve_opts* opts, ppe_solve_stats* stats, hipStream_t s);

/* ---- network (Sec. 2.4) ---- */
void ppe_net_config_default(ppe_net_config* c);
ppe_status ppe_net_create(const ppe_net_config* c, uint64_t seed, ppe_net** out); /* random init */
void ppe_net_destroy(ppe_net* n);
/* Number of FP32 parameters and the canonical flat layout (see the package's
 * Python binding for the tensor order). */
int64_t ppe_net_num_params(const ppe_net* n);
/* Copy FP32 master parameters host -> net (also refreshes the BF16 copy and
 * resets the optimiser state) or net -> host. */
ppe_status ppe_net_set_params(ppe_net* n, const float* host_params, int64_t count);
ppe_status ppe_net_get_params(const ppe_net* n, float* host_params, int64_t count);
ppe_status ppe_net_save(const ppe_net* n, const char* path);
ppe_status ppe_net_load(ppe_net* n, const char* path);

/* Forward pass on nb residual fields of one grid: y = NN(r * sqrt(N)/||r||).
 * r: device FP32 [nb][ny][nx]; y: device FP32 [nb][ny][nx]. */
ppe_status ppe_net_forward(ppe_net* n, ppe_problem* p, int32_t nb, const float* r, float* y,
                           hipStream_t s);

/* The forward on one residual field of each of count grids of any sizes
 * (Sec. 2.4), every layer as one grouped launch over the grids: each grid's
 * tiles are work items of the same launch, so small grids share the chip
 * with large ones instead of running one launch sequence each. y[i] is
 * bit-identical to ppe_net_forward on problems[i] alone.
 * problems: host array of count distinct problems (each fitting the
 * network, else PPE_ERR_SHAPE); r, y: host arrays of count device FP32
 * pointers [ny_i][nx_i]. Builds the launch tables, enqueues on stream s and
 * returns after the forwards have finished (the tables are then freed).
 * Errors: PPE_ERR_INVALID_ARG for a NULL argument, count < 0 or a repeated
 * problem; PPE_ERR_HIP. count = 0 is a no-op. */
ppe_status ppe_net_forward_batch(ppe_net* n, int32_t count, ppe_problem* const* problems, const float* const* r,
                                 float* const* y, hipStream_t s);

/* Fabricated right-hand sides on the device (stand-in for the Lanczos-Ritz
 * vectors of Eqs. 14-16): for sample s of the batch, a Gaussian random field
 * from random Fourier features (Rahimi & Recht) at the cell centres of
 * problems[s], times the cell area, minus its mean, scaled to unit RMS. The
 * random numbers are Philox4x32-10 (Salmon et al., SC 2011) with key = seed
 * and counter = (draw, s, step): draw 0 gives the sample's length scale,
 * draw 1 + f feature f (frequency by Box-Muller, phase). The same
 * (seed, step, s) always gives the same field.
 * problems: host array of nb grids of one size; R: device FP32 [nb][ny][nx].
 * Uses and synchronises stream s. */
ppe_status ppe_generate_rhs(int32_t nb, ppe_problem* const* problems, const ppe_train_opts* opts, float* R,
                            hipStream_t s);

/* Grid of fabricated training system `sample` at training step `step` (the
 * per-sample stretch and obstacle of the generator; Table 1's range of
 * stretching, an immersed obstacle as in Sec. 3). With the Philox4x32-10
 * stream of ppe_generate_rhs (key = seed, counter = (d, sample, step mod 2^32,
 * step div 2^32)) and u(x) = ((x >> 8) + 1/2) 2^-24, draw d = 0xFFFFFF00 gives
 * beta_x = 1 + 1.5 u0, beta_y = 1 + 1.5 u1 and the ellipse centre
 * (0.25 + 0.5 u2, 0.25 + 0.5 u3); draw d + 1 gives its semi-axes
 * 0.05 + 0.1 u0, 0.05 + 0.1 u1 and angle pi u2. Axes: faces
 * (1 + tanh(beta (2 i / n - 1)) / tanh beta) / 2, centres at face midpoints.
 * A cell is solid when its centre lies in the closed ellipse.
 * xc, hx: host [nx]; yc, hy: host [ny]; mask: host [ny*nx] or NULL;
 * params: host [7] or NULL (beta_x, beta_y, centre x, y, semi-axes a, b,
 * angle). Runs on the host; no device work. Errors: PPE_ERR_INVALID_ARG for
 * nx or ny < 2, more than 2^28 cells, sample < 0 or a NULL axis array. */
ppe_status ppe_generate_grid(int32_t nx, int32_t ny, uint64_t seed, uint64_t step, int32_t sample, double* xc,
                             double* yc, double* hx, double* hy, uint8_t* mask, double* params);

/* One Adam step on nb fabricated systems with the residual loss of Eq. 19,
 * Loss = mean over cells of (R - A NN(R))^2, averaged over the batch, or with
 * the supervised or A-norm loss (opts->loss_kind; see PPE_LOSS_SUPERVISED).
 * problems: host array of nb grids of one size (each sample has its own grid);
 * R: device FP32 [nb][ny][nx] (zero-sum residual fields), or NULL: the
 * library then generates the batch with ppe_generate_rhs from opts (seed,
 * step, length-scale range, features).
 * target: device FP64 [nb][ny][nx], the error fields e* of the supervised
 * and A-norm losses (required with those and an explicit R, NULL otherwise).
 * loss_out: host, the batch loss before the step. grad_out: host or NULL;
 * when given, receives the FP32 gradient that Adam uses (ppe_net_num_params
 * values; with sam_rho > 0 the one at the perturbed weights).
 * Errors: PPE_ERR_INVALID_ARG for nb outside [1, 4096] or nb x nx x ny of
 * 2^31 cells or more; PPE_ERR_SHAPE for grids of different sizes. */
ppe_status ppe_net_train_step(ppe_net* n, int32_t nb, ppe_problem* const* problems, const float* R,
                              const double* target, const ppe_train_opts* opts, float* loss_out,
                              float* grad_out, hipStream_t s);

/* ---- Lanczos-Ritz training vectors (Sec. 2.3, Eqs. 14-16) ---- */
typedef struct ppe_ritz ppe_ritz; /* opaque: Lanczos basis (device), tridiagonal and its eigen-decomposition */

/* m Lanczos steps (Eq. 14) on the grid's operator, in FP64 on the device, from
 * the start vector v0 (device FP64 [ny][nx]; its mean is removed and it is
 * normalised; the caller keeps ownership). Every step re-orthogonalises
 * against the constant null vector and all earlier Lanczos vectors (twice),
 * so the basis stays orthonormal. The tridiagonal T_m is then diagonalised
 * on the host (implicit symmetric QR, O(m^3)): ascending Ritz values theta
 * and T_m = U diag(theta) U^T. If the Krylov space is exhausted early, fewer
 * than m vectors are kept (ppe_ritz_info reports how many). Device memory:
 * (m + 1) N + m^2 doubles. 1 <= m <= min(8192, N - 1). Synchronises s.
 * Errors: PPE_ERR_INVALID_ARG (bad m, or a zero or constant v0),
 * PPE_ERR_NONFINITE, PPE_NOT_CONVERGED (eigen-decomposition), PPE_ERR_HIP. */
ppe_status ppe_ritz_create(ppe_problem* p, int32_t m, const double* v0, ppe_ritz** out, hipStream_t s);
/* Kept size m and host copies of alpha [m], beta [m - 1] and theta [m]
 * (ascending); any pointer may be NULL. */
ppe_status ppe_ritz_info(const ppe_ritz* r, int32_t* m, double* alpha, double* beta, double* theta);
/* nb training vectors R^i = scale Q c^i / |Q c^i|_2 (Eq. 15 for scale = 1;
 * scale = sqrt(N) gives unit RMS, the scale of the random-field data), Q = V_m U the Ritz
 * vectors in ascending order, c^i_j = 9 N(0,1) for j <= b m and N(0,1)
 * otherwise (Eq. 16). Normal draws: Philox4x32-10, key = seed, counter =
 * (j, i + 2^31, step mod 2^32, step div 2^32), Box-Muller; each Ritz vector
 * is signed so that its component along v_0 is not negative. R: device FP32
 * [nb][ny][nx]. 1 <= nb <= 4096, 0 <= b <= 1. Synchronises s. */
ppe_status ppe_ritz_rhs(const ppe_ritz* r, int32_t nb, uint64_t seed, int64_t step, double b, double scale,
                        float* R, hipStream_t s);
void ppe_ritz_destroy(ppe_ritz* r);
/* Host-only: eigenvalues (ascending, theta [n]) and eigenvectors (U [n][n],
 * row-major, column j = eigenvector j, signed so that U[0][j] >= 0; may be
 * NULL) of the symmetric tridiagonal matrix with diagonal alpha [n] and
 * off-diagonal beta [n - 1]. */
ppe_status ppe_tridiag_eigh(int32_t n, const double* alpha, const double* beta, double* theta, double* U);

/* ---- measurement ---- */
/* Launch-configuration tuning of the plain solve (per problem and batch
 * size nb). ppe_tune_pcg runs every iteration form x tile height (2, 4, 8,
 * 16 rows per wavefront) for `reps` iterations on the caller's system
 * (f: device FP32 [nb][ny][nx]; x: device FP64 [nb][ny][nx], overwritten),
 * timing each launch with HIP events, and stores the fastest in the problem
 * (the untuned default stays unless another candidate is more than 3 %
 * faster); later solves with variant PPE_PCG_AUTO and rows_per_wave 0 use it.
 * out (host, optional) receives the choice and the per-iteration times in
 * microseconds (per CG iteration: a two-step launch counts as two),
 * us_per_iter[form][k] for form 0 single reduction, 1 two-phase, 2 two-step
 * and k indexing the heights 2, 4, 8, 16, 20, 24 (0 where the form has no
 * such height: 20 and 24 are built for the two-step form only). ppe_set_tuning stores a
 * choice directly (e.g. from a cache the caller keeps); ppe_get_tuning
 * reports what PPE_PCG_AUTO resolves to for nb. */
typedef struct {
  int32_t variant, rows_per_wave;
  double us_per_iter[3][6];
} ppe_tune_result;
ppe_status ppe_tune_pcg(ppe_problem* p, int32_t nb, const float* f, double* x, int32_t reps,
                        ppe_tune_result* out, hipStream_t s);
ppe_status ppe_set_tuning(ppe_problem* p, int32_t nb, int32_t variant, int32_t rows_per_wave);

/* Launch-configuration tuning of the network forward (the Sec. 2.4 network)
 * on one grid, per problem, network and batch size nb: every 3x3 or 1x1
 * up-convolution with at least 64 output channels can run with 32 or 64
 * output channels per workgroup (more workgroups and occupancy, or fewer
 * re-reads of the input). By default a layer takes 64 when that still gives
 * at least two workgroups per compute unit, else 32. ppe_tune_net runs the
 * forward once on nb zero fields, then times each such launch `reps` times
 * (HIP events) with either width and keeps the default unless the other is
 * more than 3 % faster; later forwards of this problem with this network use
 * the choice (a tile width can change a layer's K split, so outputs may
 * differ from the untuned ones in rounding). In the grouped forward of a
 * mixed-size batch each grid keeps the K split of its own (tuned or default)
 * width, so its result stays bit-identical. The choice is dropped when the
 * problem's network buffers are rebuilt (another network or a larger nb).
 * out (host, optional): n = launches of one forward; for launch k the chosen
 * width (0 where there is no choice) and the measured microseconds per
 * launch with either width (0 where not timed). reps in [1, 1000]. */
#define PPE_NET_MAX_LAUNCHES 64
typedef struct {
  int32_t n;
  int32_t tile[PPE_NET_MAX_LAUNCHES];
  float us32[PPE_NET_MAX_LAUNCHES];
  float us64[PPE_NET_MAX_LAUNCHES];
} ppe_net_tune_result;
ppe_status ppe_tune_net(ppe_net* n, ppe_problem* p, int32_t nb, int32_t reps, ppe_net_tune_result* out,
                        hipStream_t s);
ppe_status ppe_get_tuning(const ppe_problem* p, int32_t nb, int32_t* variant, int32_t* rows_per_wave);

/* Average kernel durations in ms of the PCG iteration on nb systems, for the
 * form opts->variant selects: TWO_PHASE gives one phase-A launch in ms_out[0]
 * and one phase-B launch in ms_out[1]; SINGLE_REDUCTION and TWO_STEP give
 * one launch (one, resp. two iterations) in ms_out[0] and 0 in ms_out[1]. After a solve setup on
 * (f, x), `reps` iterations run eagerly on stream s, as in a solve,
 * each launch carrying its own start/stop HIP events (hipExtLaunchKernelGGL),
 * so the elapsed times are kernel execution times. x is used as the
 * initial guess and its content is left unspecified. ms_out: host [2]. */
ppe_status ppe_profile_pcg(ppe_problem* p, int32_t nb, const float* f, double* x,
                           const ppe_solve_opts* opts, int32_t reps, double* ms_out, hipStream_t s);
/* Average ms of a plain device copy of `bytes` bytes (multiple of 16) from src
 * to dst (device buffers, caller-owned): the bandwidth reference and the
 * calibration kernel for hardware byte counters. ms_out: host [1]. */
ppe_status ppe_profile_copy(const void* src, void* dst, int64_t bytes, int32_t reps, double* ms_out,
                            hipStream_t s);

/* ---- allocation-free plain solve ----
 * For callers that cannot allocate device memory while they run (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the Jacobi-PCG / CG solve of ppe_solve_plain for ONE right-hand side, with
 * its solver state (six FP32 vectors, FP64 partial sums, iteration state) in
 * a fixed device array of PPE_NOALLOC_SCRATCH_BYTES bytes that the library
 * holds on every device it runs on until the process ends. The call makes no
 * device or pinned-host allocation and frees nothing: it launches the solve's
 * kernels eagerly on stream s (no HIP graph) and polls convergence with
 * synchronous device-to-host copies into host stack memory. The kernels and
 * their order are those of ppe_solve_plain with the same iteration form and
 * tile height, so the result is bit-identical to that call's.
 * p, opts, stats: as for ppe_solve_plain with nb = 1 (the problem's
 * workspace is not touched). f: device FP32 [ny][nx]; x: device FP64
 * [ny][nx], in = initial guess (unless opts->zero_x0), out = zero-mean
 * solution.
 * The grid's state must fit the array: ppe_noalloc_scratch_bytes(p) bytes,
 * about 24 bytes per cell plus the partial sums (a 1024 x 1024 grid needs
 * 26 MB). A larger grid gives PPE_ERR_INVALID_ARG before anything is
 * launched. All calls on one device share its array, which keeps the last
 * call's contents (each call clears what must start at zero): the library
 * serialises calls within a process with a lock, and a caller must not
 * overlap a call with another use of the same device's array. */
#define PPE_NOALLOC_SCRATCH_BYTES (32 * 1024 * 1024)
int64_t ppe_noalloc_scratch_bytes(const ppe_problem* p); /* -1 for NULL */
ppe_status ppe_solve_plain_noalloc(const ppe_problem* p, const float* f, double* x, const ppe_solve_opts* opts,
                                   ppe_solve_stats* stats, hipStream_t s);

const char* ppe_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PPE_H */
