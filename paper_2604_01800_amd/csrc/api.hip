// C-ABI and host runtime of the MI355X PPE library: problem handles,
// workspaces, graph-captured PCG iteration chunks and convergence polling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ppe.h"
#include "api_internal.hpp"
#include "kernels.hpp"
#include "mg_internal.hpp"

namespace ppe {

thread_local std::string g_last_error;

ppe_status set_error(ppe_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

void* dev_alloc(size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 256;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

void dev_free(void* p) {
  if (p) (void)hipFree(p);
}

static void free_ws(SolveWs& w) {
  if (w.exec) (void)hipGraphExecDestroy(w.exec);
  w.exec = nullptr;
  dev_free(w.vec);
  dev_free(w.part);
  dev_free(w.st);
  dev_free(w.flags);
  dev_free(w.call);
  dev_free(w.hist);
  if (w.h_flags) (void)hipHostFree(w.h_flags);
  if (w.h_state) (void)hipHostFree(w.h_state);
  for (auto& e : w.ev)
    if (e) (void)hipEventDestroy(e);
  w = SolveWs{};
}

// Workspace for nb solves: 6 FP32 vectors per solve (x_c, r, p0, p1, e, r1),
// the partial-sum arrays (16 per workgroup and solve of the 64-column tiles,
// then 22 per workgroup and solve of the two-iteration form's 56-column
// tiles), states and polling flags.
ppe_status ensure_ws(ppe_problem* p, int nb) {
  SolveWs& w = p->ws;
  if (w.nb >= nb && w.vec) return PPE_OK;
  free_ws(w);
  const int64_t N = (int64_t)p->nx * p->ny;
  ws_extent(p, &w.Pmax, &w.P2max);
  w.vec = (float*)dev_alloc(sizeof(float) * 6 * N * nb);
  w.part = (double*)dev_alloc(sizeof(double) * (16 * (size_t)w.Pmax + 22 * (size_t)w.P2max) * nb);
  w.st = (SolveState*)dev_alloc(sizeof(SolveState) * nb);
  w.flags = (int32_t*)dev_alloc(sizeof(int32_t) * nb);
  w.call = (CallArgs*)dev_alloc(sizeof(CallArgs));
  if (!w.vec || !w.part || !w.st || !w.flags || !w.call) {
    free_ws(w);
    return set_error(PPE_ERR_HIP, "device allocation of the solve workspace (%d x %lld cells) failed", nb,
                     (long long)N);
  }
  if (hipHostMalloc((void**)&w.h_flags, sizeof(int32_t) * 2 * nb, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&w.h_state, sizeof(SolveState) * nb, hipHostMallocDefault) != hipSuccess) {
    free_ws(w);
    return set_error(PPE_ERR_HIP, "pinned host allocation failed");
  }
  for (auto& e : w.ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      free_ws(w);
      return set_error(PPE_ERR_HIP, "hipEventCreate failed");
    }
  w.nb = nb;
  return PPE_OK;
}

PcgArgs make_pcg_args_at(const ppe_problem* p, const WsView& w, int nb, int R, int jacobi, double tol, int tol_kind,
                         int zero_x0) {
  PcgArgs a{};
  a.c = p->coef;
  const dim3 g = stencil_grid(p->coef, R, 1);
  a.P = (int)(g.x * g.y);
  a.R = R;
  a.N = (int64_t)p->nx * p->ny;
  const size_t N = (size_t)a.N * nb;
  a.xc = w.vec;
  a.r = w.vec + N;
  a.p0 = w.vec + 2 * N;
  a.p1 = w.vec + 3 * N;
  a.partA = w.part;
  a.partB = w.part + (size_t)a.P * nb;
  a.partD = w.part + (size_t)3 * a.P * nb;
  a.e = w.vec + 4 * N;
  a.r1 = w.vec + 5 * N;
  a.part1 = w.part + (size_t)6 * a.P * nb;
  a.P2 = (int)stencil_grid2(p->coef, R, 1).x;
  a.part2 = w.part + (size_t)16 * w.Pmax * nb;
  a.st = w.st;
  a.flags = w.flags;
  a.call = w.call;
  a.tol = tol;
  a.tol_kind = tol_kind;
  a.jacobi = jacobi;
  a.zero_x0 = zero_x0;
  return a;
}

void ws_extent(const ppe_problem* p, int* Pmax, int* P2max) {
  const dim3 g = stencil_grid(p->coef, 2, 1);  // the smallest tile height has the most workgroups
  *Pmax = (int)(g.x * g.y);
  *P2max = (int)stencil_grid2(p->coef, 2, 1).x;
}

PcgArgs make_pcg_args(ppe_problem* p, int nb, int R, int jacobi, double tol, int tol_kind, int zero_x0) {
  SolveWs& w = p->ws;
  const WsView v{w.vec, w.part, w.Pmax, w.st, w.flags, w.call};
  return make_pcg_args_at(p, v, nb, R, jacobi, tol, tol_kind, zero_x0);
}

int default_rows(const ppe_problem* p, int nb) {
  // Enough workgroups to cover the 256 CUs several times over.
  const int64_t cells = (int64_t)p->nx * p->ny * nb;
  if (cells >= (int64_t)4 << 20) return 16;
  if (cells >= (int64_t)1 << 20) return 8;
  if (cells >= (int64_t)1 << 17) return 4;
  return 2;
}

static int default_rows_single(int64_t cells) {
  if (cells >= (int64_t)1 << 20) return 16;
  if (cells >= (int64_t)1 << 18) return 8;
  if (cells >= (int64_t)1 << 16) return 4;
  return 2;
}

// Tile heights (rows per wavefront) built for each iteration form.
bool height_ok(int form, int R) {
  if (R == 2 || R == 4 || R == 8 || R == 16) return true;
  return form == PPE_PCG_TWO_STEP && (R == 20 || R == 24);
}

// Number of compute units of the current device (256 on MI355X).
static int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      cus = n;
    else
      cus = 256;
  }
  return cus;
}

// Two-step form: the launch is bound by the instruction stream of its
// busiest CU, about (workgroups per CU, rounded up) x (rows per wavefront +
// the 8 halo rows); take the height that minimises that over the launch's
// workgroups (nb solves on each of the n grids).
int default_rows_two_step(const ppe_problem* const* probs, int n, int nb) {
  static const int kH[6] = {2, 4, 8, 16, 20, 24};
  int best = 2;
  int64_t best_cost = INT64_MAX;
  for (int R : kH) {
    int64_t wg = 0;
    for (int i = 0; i < n; ++i) wg += (int64_t)stencil_grid2(probs[i]->coef, R, 1).x * nb;
    const int64_t cost = ((wg + device_cus() - 1) / device_cus()) * (R + 8);
    if (cost < best_cost) {
      best_cost = cost;
      best = R;
    }
  }
  return best;
}

void resolve_plain(const ppe_problem* p, int nb, const ppe_solve_opts& o, int* form, int* rows) {
  const int64_t cells = (int64_t)p->nx * p->ny * nb;
  int v = o.variant, R = o.rows_per_wave;
  if (v == PPE_PCG_AUTO) {
    for (const auto& t : p->tuned)
      if (t[0] == nb) {
        v = t[1];
        if (R == 0) R = t[2];
      }
  }
  if (v == PPE_PCG_AUTO) v = PPE_PCG_TWO_STEP;
  // the multigrid preconditioner, masked operators and residual histories
  // are built on the two-phase iteration
  if (o.precond == PPE_PC_MG || o.precond == PPE_PC_IC || o.record_history || p->mask_mode == PPE_MASK_SOLID) {
    if (v != PPE_PCG_TWO_PHASE) R = 0;
    v = PPE_PCG_TWO_PHASE;
  }
  *form = v;
  if (!height_ok(v, R))
    R = v == PPE_PCG_TWO_PHASE ? default_rows(p, nb)
        : v == PPE_PCG_TWO_STEP ? default_rows_two_step(&p, 1, nb)
                                : default_rows_single(cells);
  *rows = R;
}

int rows_of(const ppe_problem* p, int nb, const ppe_solve_opts& o) {
  const int r = o.rows_per_wave;
  if (r == 2 || r == 4 || r == 8 || r == 16) return r;
  return default_rows(p, nb);
}

#define HIPCHK(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return set_error(PPE_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));      \
  } while (0)

// One chunk of `chunk` launches with alternating parity: pairs of phase
// launches (two-phase form) or single launches (single-reduction and
// two-step forms).
void launch_chunk(const PcgArgs& a, int nb, int chunk, int form, hipStream_t s) {
  for (int k = 0; k < chunk; ++k) {
    if (form == PPE_PCG_SINGLE_REDUCTION) launch_pcg1_step(a, nb, k & 1, s);
    else if (form == PPE_PCG_TWO_STEP) launch_pcg2_step(a, nb, k & 1, s);
    else launch_pcg_pair(a, nb, k & 1, 0, 0, s);
  }
}

// Capture (once per workspace shape and iteration form) the chunk as a graph.
static ppe_status get_chunk_graph(ppe_problem* p, const PcgArgs& a, int nb, int chunk, int form) {
  SolveWs& w = p->ws;
  const std::array<int64_t, 8> key = {nb, a.R, a.jacobi + (a.icq ? 2 : 0), chunk, form,
                                      a.mg ? (int64_t)a.mg->uid : 0, (int64_t)(intptr_t)a.hist, a.hist_cap};
  if (w.exec && key == w.exec_key) return PPE_OK;
  if (w.exec) {
    (void)hipGraphExecDestroy(w.exec);
    w.exec = nullptr;
  }
  if (!p->cap_stream) HIPCHK(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  HIPCHK(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
  launch_chunk(a, nb, chunk, form, p->cap_stream);
  hipError_t e = hipStreamEndCapture(p->cap_stream, &graph);
  if (e != hipSuccess) return set_error(PPE_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&w.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    w.exec = nullptr;
    return set_error(PPE_ERR_HIP, "graph instantiate failed: %s", hipGetErrorString(e));
  }
  w.exec_key = key;
  return PPE_OK;
}

// Replays iteration chunks until every solve of the batch has finished. The
// next chunk is enqueued before the previous chunk's flags are inspected, so
// the device never waits for the host.
ppe_status run_pcg_chunks(ppe_problem* p, const PcgArgs& a, int nb, const ppe_solve_opts& o, hipStream_t s,
                          int form) {
  SolveWs& w = p->ws;
  // Iterations per polled chunk: multigrid converges in tens of iterations,
  // Jacobi-PCG in thousands; a chunk may run past convergence by up to two
  // chunks of early-exit launches.
  int chunk = o.chunk > 0 ? o.chunk : (a.mg ? 8 : a.icq ? 32 : 64);
  chunk += chunk & 1;
  if (o.use_graph) {
    ppe_status st = get_chunk_graph(p, a, nb, chunk, form);
    if (st != PPE_OK) return st;
  }
  // Launches a solve can take: a CG iteration is one pair (two-phase) or at
  // most one launch (single reduction, two-step), a reliable update one pair
  // or three launches.
  const int64_t max_chunks = (3 * (int64_t)o.max_iter + 8) / chunk + 2;
  for (int64_t c = 0; c < max_chunks; ++c) {
    if (o.use_graph) {
      HIPCHK(hipGraphLaunch(w.exec, s));
    } else {
      launch_chunk(a, nb, chunk, form, s);
      HIPCHK(hipGetLastError());
    }
    HIPCHK(hipMemcpyAsync(w.h_flags + (c & 1) * nb, w.flags, sizeof(int32_t) * nb,
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(w.ev[c & 1], s));
    if (c >= 1) {
      HIPCHK(hipEventSynchronize(w.ev[(c - 1) & 1]));
      const int32_t* fl = w.h_flags + ((c - 1) & 1) * nb;
      bool all = true;
      for (int i = 0; i < nb; ++i) all = all && fl[i] != DONE_NO;
      if (all) return PPE_OK;
    }
  }
  return PPE_OK;
}

// Rate of the device real-time clock (wall_clock64) in kHz.
double wall_clock_khz() {
  static double khz = 0.0;
  if (khz == 0.0) {
    int dev = 0, rate = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, dev) == hipSuccess && rate > 0)
      khz = (double)rate;
    else
      khz = 1e5;  // the documented 100 MHz counter
  }
  return khz;
}

void stats_from_state(const SolveState& S, ppe_status st, double ms, bool hybrid, ppe_solve_stats* out) {
  ppe_solve_stats& o = *out;
  memset(&o, 0, sizeof o);
  o.status = st;
  o.iters_total = S.it_final;
  o.iters_cg = S.itcg_final;
  o.iters_dlsm = hybrid ? S.n_dlsm : 0;
  o.dlsm_rejected = hybrid ? S.n_rej : 0;
  o.reliable_updates = S.nru_final;
  o.abs_res_true = std::sqrt(S.rr_final);
  o.bnorm = std::sqrt(S.bnorm2);
  o.rel_res_true = S.bnorm2 > 0 ? std::sqrt(S.rr_final / S.bnorm2) : o.abs_res_true;
  o.rhs_mean_removed = S.bmean;
  o.ms_total = ms;
  o.ms_device = (double)(S.t_done - S.t_start) / wall_clock_khz();
}

ppe_status state_status(const SolveState& S) {
  return S.done == DONE_CONV ? PPE_OK : S.done == DONE_NONFINITE ? PPE_ERR_NONFINITE : PPE_NOT_CONVERGED;
}

// The red-black IC(0) diagonals of a problem (FP64 on the host, rounded
// once): q = 1/D on red cells, 1/S_b on black cells with
// S_b = D_b - sum over the red neighbours r of w_br^2 / D_r; and its output
// buffer for nb right-hand sides.
static ppe_status ic_ensure(ppe_problem* p, int nb, hipStream_t s) {
  const int nx = p->nx, ny = p->ny;
  const int64_t N = (int64_t)nx * ny;
  if (!p->d_icq) {
    std::vector<double> gx(nx + 1, 0.0), gy(ny + 1, 0.0);
    for (int k = 1; k < nx; ++k) gx[k] = 1.0 / (p->xc[k] - p->xc[k - 1]);
    for (int k = 1; k < ny; ++k) gy[k] = 1.0 / (p->yc[k] - p->yc[k - 1]);
    auto D = [&](int i, int j) { return p->hy[j] * (gx[i] + gx[i + 1]) + p->hx[i] * (gy[j] + gy[j + 1]); };
    std::vector<float> q((size_t)N);
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double d = D(i, j);
        if ((i + j) % 2) {  // black: the four red neighbours (face weight 0 at a wall)
          if (i > 0) d -= std::pow(p->hy[j] * gx[i], 2) / D(i - 1, j);
          if (i + 1 < nx) d -= std::pow(p->hy[j] * gx[i + 1], 2) / D(i + 1, j);
          if (j > 0) d -= std::pow(p->hx[i] * gy[j], 2) / D(i, j - 1);
          if (j + 1 < ny) d -= std::pow(p->hx[i] * gy[j + 1], 2) / D(i, j + 1);
        }
        if (!(d > 0.0)) return set_error(PPE_ERR_SHAPE, "IC(0) breaks down at cell (%d, %d)", i, j);
        q[(size_t)j * nx + i] = (float)(1.0 / d);
      }
    float* dq = (float*)dev_alloc(sizeof(float) * N);
    if (!dq) return set_error(PPE_ERR_HIP, "allocation of the IC(0) diagonals failed");
    const hipError_t e = hipMemcpyAsync(dq, q.data(), sizeof(float) * N, hipMemcpyHostToDevice, s);
    const hipError_t es = hipStreamSynchronize(s);  // q goes out of scope
    if (e != hipSuccess || es != hipSuccess) {
      dev_free(dq);
      return set_error(PPE_ERR_HIP, "upload of the IC(0) diagonals failed");
    }
    p->d_icq = dq;
  }
  if (p->ic_nb < nb) {
    dev_free(p->d_icz);
    p->d_icz = (float*)dev_alloc(sizeof(float) * N * nb);
    p->ic_nb = p->d_icz ? nb : 0;
    if (!p->d_icz) return set_error(PPE_ERR_HIP, "allocation of the IC(0) output failed");
  }
  return PPE_OK;
}

ppe_status attach_extras(ppe_problem* p, PcgArgs& a, int nb, const ppe_solve_opts& o, hipStream_t s) {
  if (o.precond == PPE_PC_IC) {
    ppe_status st = ic_ensure(p, nb, s);
    if (st != PPE_OK) return st;
    a.icq = p->d_icq;
    a.z = p->d_icz;
    a.jacobi = 0;
  }
  if (o.precond == PPE_PC_MG) {
    ppe_status st = mg_ensure(p, o.mg_levels > 0 ? o.mg_levels : 4, nb, a.R, s);
    if (st != PPE_OK) return st;
    a.mg = p->mg;
    a.z = p->mg->z;
    a.jacobi = 0;
  }
  if (o.record_history) {
    SolveWs& w = p->ws;
    const int cap = (int)std::min<int64_t>((int64_t)o.max_iter + 1, (int64_t)1 << 22);
    const int64_t need = (int64_t)cap * nb;
    if (w.hist_elems < need) {
      if (w.exec) {  // a captured graph may hold the old buffer
        (void)hipGraphExecDestroy(w.exec);
        w.exec = nullptr;
      }
      dev_free(w.hist);
      w.hist = (double*)dev_alloc(sizeof(double) * need);
      w.hist_elems = w.hist ? need : 0;
      if (!w.hist) return set_error(PPE_ERR_HIP, "allocation of the residual histories failed");
    }
    a.hist = w.hist;
    a.hist_cap = cap;
  }
  return PPE_OK;
}

ppe_status fill_stats(ppe_problem* p, int nb, ppe_solve_stats* stats, double ms, hipStream_t s, bool hybrid,
                      const PcgArgs& a) {
  SolveWs& w = p->ws;
  HIPCHK(hipMemcpyAsync(w.h_state, a.st, sizeof(SolveState) * nb, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  ppe_status worst = PPE_OK;
  const double khz = wall_clock_khz();
  for (int i = 0; i < nb; ++i) {
    const SolveState& S = w.h_state[i];
    const ppe_status st = state_status(S);
    if (st == PPE_ERR_NONFINITE) worst = st;
    else if (st == PPE_NOT_CONVERGED && worst == PPE_OK) worst = st;
    if (!stats) continue;
    ppe_solve_stats& o = stats[i];
    double* hbuf = o.history;
    const int hcap = o.history_cap;
    stats_from_state(S, st, ms, hybrid, &o);
    if (hybrid) {
      // the phase clocks run on the first solve's state, for the whole call
      const SolveState& S0 = w.h_state[0];
      o.ms_pcg = (double)S0.t_acc[0] / khz;
      o.ms_net = (double)S0.t_acc[1] / khz;
      o.ms_dlsm = (double)S0.t_acc[2] / khz;
    } else {
      o.ms_pcg = o.ms_device;
    }
    o.history = hbuf;
    o.history_cap = hcap;
    if (a.hist && hbuf && hcap > 0) {
      const int n = std::min(std::min(hcap, a.hist_cap), S.it_final + 1);
      if (n > 0)
        HIPCHK(hipMemcpy(hbuf, a.hist + (size_t)i * a.hist_cap, sizeof(double) * n, hipMemcpyDeviceToHost));
      o.history_len = std::max(n, 0);
    }
  }
  if (worst == PPE_ERR_NONFINITE) set_error(worst, "non-finite value in a source field or iteration");
  return worst;
}

ppe_status check_solve_args(const ppe_problem* p, int32_t nb, const void* f, const void* x,
                            const ppe_solve_opts* opts) {
  if (!p) return set_error(PPE_ERR_INVALID_ARG, "problem is NULL");
  if (nb < 0) return set_error(PPE_ERR_INVALID_ARG, "nb < 0");
  if (nb > 65535) return set_error(PPE_ERR_INVALID_ARG, "nb > 65535");
  if (nb > 0 && (!f || !x)) return set_error(PPE_ERR_INVALID_ARG, "f or x is NULL");
  if (opts) {
    if (!(opts->tol >= 0.0) || !std::isfinite(opts->tol))
      return set_error(PPE_ERR_INVALID_ARG, "tol must be finite and >= 0");
    if (opts->max_iter < 0) return set_error(PPE_ERR_INVALID_ARG, "max_iter < 0");
    if (opts->precond != PPE_PC_NONE && opts->precond != PPE_PC_JACOBI && opts->precond != PPE_PC_MG &&
        opts->precond != PPE_PC_IC)
      return set_error(PPE_ERR_INVALID_ARG, "unknown preconditioner %d", opts->precond);
    if (p->mask_mode == PPE_MASK_SOLID && (opts->precond == PPE_PC_MG || opts->precond == PPE_PC_IC))
      return set_error(PPE_ERR_UNSUPPORTED, "the multigrid and IC preconditioners do not take PPE_MASK_SOLID grids");
    if (opts->precond == PPE_PC_IC && (p->nx < 2 || p->ny < 2))
      return set_error(PPE_ERR_SHAPE, "the IC(0) preconditioner needs nx and ny of at least 2 (got %d x %d)", p->nx,
                       p->ny);
    if (opts->mg_levels < 0 || opts->mg_levels > 12)
      return set_error(PPE_ERR_INVALID_ARG, "mg_levels must lie in [0, 12]");
    if (opts->precond == PPE_PC_MG) {
      const int L = opts->mg_levels ? opts->mg_levels : 4;
      if (p->nx % (1 << (L - 1)) || p->ny % (1 << (L - 1)))
        return set_error(PPE_ERR_SHAPE, "multigrid with %d levels needs nx, ny divisible by %d (got %d x %d)", L,
                         1 << (L - 1), p->nx, p->ny);
    }
    if (opts->tol_kind != PPE_TOL_RELATIVE && opts->tol_kind != PPE_TOL_ABSOLUTE)
      return set_error(PPE_ERR_INVALID_ARG, "tol_kind %d", opts->tol_kind);
    if (!(opts->reliable_delta > 0.0 && opts->reliable_delta < 1.0))
      return set_error(PPE_ERR_INVALID_ARG, "reliable_delta must lie in (0, 1)");
  }
  return PPE_OK;
}

ppe_status reject_solid(const ppe_problem* p, const char* what) {
  if (p && p->mask_mode == PPE_MASK_SOLID)
    return set_error(PPE_ERR_UNSUPPORTED, "%s does not take PPE_MASK_SOLID grids", what);
  return PPE_OK;
}

void launch_setup(const PcgArgs& a, int nb, int form, hipStream_t s) {
  if (form == PPE_PCG_SINGLE_REDUCTION) launch_pcg1_setup(a, nb, s);
  else if (form == PPE_PCG_TWO_STEP) launch_pcg2_setup(a, nb, s);
  else launch_pcg_setup(a, nb, s);
}

ppe_status solve_plain_impl(ppe_problem* p, int32_t nb, const float* f, double* x,
                            const ppe_solve_opts& o, ppe_solve_stats* stats, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  ppe_status st = ensure_ws(p, nb);
  if (st != PPE_OK) return st;
  int form, R;
  resolve_plain(p, nb, o, &form, &R);
  PcgArgs a = make_pcg_args(p, nb, R, o.precond == PPE_PC_JACOBI, o.tol, o.tol_kind, o.zero_x0);
  st = attach_extras(p, a, nb, o, s);
  if (st != PPE_OK) return st;
  launch_set_call(p->ws.call, f, x, o.max_iter, o.reliable_delta * o.reliable_delta, s);
  launch_setup(a, nb, form, s);
  HIPCHK(hipGetLastError());
  st = run_pcg_chunks(p, a, nb, o, s, form);
  if (st != PPE_OK) return st;
  launch_pcg_finish(a, nb, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return fill_stats(p, nb, stats, ms, s, false, a);
}

// Average kernel durations of `reps` iterations of one launch configuration
// (setup first), each launch carrying its own start/stop events.
ppe_status profile_form(ppe_problem* p, int nb, const float* f, double* x, const ppe_solve_opts& o, int form,
                        int R, int reps, double* ms_out, hipStream_t s) {
  ppe_status st = ensure_ws(p, nb);
  if (st != PPE_OK) return st;
  PcgArgs a = make_pcg_args(p, nb, R, o.precond == PPE_PC_JACOBI, o.tol, o.tol_kind, o.zero_x0);
  st = attach_extras(p, a, nb, o, s);
  if (st != PPE_OK) return st;
  launch_set_call(p->ws.call, f, x, o.max_iter, o.reliable_delta * o.reliable_delta, s);
  launch_setup(a, nb, form, s);
  const bool single = form != PPE_PCG_TWO_PHASE;
  std::vector<hipEvent_t> ev(4 * reps);
  for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  for (int k = 0; k < reps; ++k) {
    if (form == PPE_PCG_SINGLE_REDUCTION) {
      launch_pcg1_step_timed(a, nb, 0, s, ev[4 * k], ev[4 * k + 1]);
      launch_pcg1_step_timed(a, nb, 1, s, ev[4 * k + 2], ev[4 * k + 3]);
    } else if (form == PPE_PCG_TWO_STEP) {
      launch_pcg2_step_timed(a, nb, 0, s, ev[4 * k], ev[4 * k + 1]);
      launch_pcg2_step_timed(a, nb, 1, s, ev[4 * k + 2], ev[4 * k + 3]);
    } else {
      launch_pcg_phase_timed(a, nb, k & 1, 0, s, ev[4 * k], ev[4 * k + 1]);
      launch_pcg_phase_timed(a, nb, k & 1, 1, s, ev[4 * k + 2], ev[4 * k + 3]);
    }
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventSynchronize(ev[4 * reps - 1]));
  double ta = 0, tb = 0;
  for (int k = 0; k < reps; ++k) {
    float t1 = 0, t2 = 0;
    HIPCHK(hipEventElapsedTime(&t1, ev[4 * k], ev[4 * k + 1]));
    HIPCHK(hipEventElapsedTime(&t2, ev[4 * k + 2], ev[4 * k + 3]));
    ta += t1;
    tb += t2;
  }
  if (single) {
    ms_out[0] = (ta + tb) / (2.0 * reps);
    ms_out[1] = 0.0;
  } else {
    ms_out[0] = ta / reps;
    ms_out[1] = tb / reps;
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  return PPE_OK;
}

}  // namespace ppe

using namespace ppe;

extern "C" {

const char* ppe_last_error(void) { return g_last_error.c_str(); }

void ppe_solve_opts_default(ppe_solve_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof *o);
  o->tol = 1e-6;
  o->tol_kind = PPE_TOL_RELATIVE;
  o->precond = PPE_PC_JACOBI;
  o->max_iter = 100000;
  o->num_cg = 3;
  o->num_dlsm = 2;
  o->direction = PPE_DIR_NET;
  o->reliable_delta = 0.3;
  o->rows_per_wave = 0;
  o->use_graph = 1;
  o->chunk = 0;
  o->variant = PPE_PCG_AUTO;
}

ppe_status ppe_problem_create(const ppe_grid_desc* g, hipStream_t s, ppe_problem** out) {
  if (!g || !out) return set_error(PPE_ERR_INVALID_ARG, "grid or out is NULL");
  *out = nullptr;
  const int nx = g->nx, ny = g->ny;
  if (nx < 2 || ny < 2) return set_error(PPE_ERR_SHAPE, "nx, ny must be >= 2 (got %d x %d)", nx, ny);
  if ((int64_t)nx * ny > ((int64_t)1 << 28)) return set_error(PPE_ERR_SHAPE, "grid too large (at most 2^28 cells)");
  if (!g->xc || !g->yc || !g->hx || !g->hy) return set_error(PPE_ERR_INVALID_ARG, "NULL coordinate array");
  for (int i = 0; i < nx; ++i) {
    if (!std::isfinite(g->xc[i]) || !(g->hx[i] > 0.0) || !std::isfinite(g->hx[i]))
      return set_error(PPE_ERR_INVALID_ARG, "xc/hx invalid at i=%d", i);
    if (i > 0 && !(g->xc[i] > g->xc[i - 1])) return set_error(PPE_ERR_INVALID_ARG, "xc not increasing at %d", i);
  }
  for (int j = 0; j < ny; ++j) {
    if (!std::isfinite(g->yc[j]) || !(g->hy[j] > 0.0) || !std::isfinite(g->hy[j]))
      return set_error(PPE_ERR_INVALID_ARG, "yc/hy invalid at j=%d", j);
    if (j > 0 && !(g->yc[j] > g->yc[j - 1])) return set_error(PPE_ERR_INVALID_ARG, "yc not increasing at %d", j);
  }
  static std::atomic<uint64_t> next_uid{1};
  if (g->mask_mode != PPE_MASK_DIBPM && g->mask_mode != PPE_MASK_SOLID)
    return set_error(PPE_ERR_INVALID_ARG, "mask_mode %d", g->mask_mode);
  if (g->mask_mode == PPE_MASK_SOLID) {
    if (!g->mask) return set_error(PPE_ERR_INVALID_ARG, "PPE_MASK_SOLID needs a mask");
    int64_t fluid = 0;
    for (int64_t k = 0; k < (int64_t)nx * ny; ++k) fluid += g->mask[k] == 0;
    if (fluid == 0) return set_error(PPE_ERR_INVALID_ARG, "PPE_MASK_SOLID needs at least one fluid cell");
  }
  ppe_problem* p = new ppe_problem();
  p->uid = next_uid.fetch_add(1);
  p->nx = nx;
  p->ny = ny;
  p->xc.assign(g->xc, g->xc + nx);
  p->yc.assign(g->yc, g->yc + ny);
  p->hx.assign(g->hx, g->hx + nx);
  p->hy.assign(g->hy, g->hy + ny);
  if (g->mask) p->mask.assign(g->mask, g->mask + (size_t)nx * ny);
  p->mask_mode = g->mask_mode;
  ppe_status st = problem_upload(p, s);
  if (st != PPE_OK) {
    ppe_problem_destroy(p);
    return st;
  }
  *out = p;
  return PPE_OK;
}

void ppe_problem_destroy(ppe_problem* p) {
  if (!p) return;
  free_ws(p->ws);
  problem_release(p);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  delete p;
}

ppe_status ppe_apply_f32(const ppe_problem* p, int32_t nb, const float* x, float* y, hipStream_t s) {
  if (!p || nb < 0 || (nb > 0 && (!x || !y))) return set_error(PPE_ERR_INVALID_ARG, "bad arguments");
  if (nb == 0) return PPE_OK;
  launch_apply_f32(p->coef, nb, x, y, 4, s);
  HIPCHK(hipGetLastError());
  return PPE_OK;
}

ppe_status ppe_apply_f64(const ppe_problem* p, int32_t nb, const double* x, double* y, hipStream_t s) {
  if (!p || nb < 0 || (nb > 0 && (!x || !y))) return set_error(PPE_ERR_INVALID_ARG, "bad arguments");
  if (nb == 0) return PPE_OK;
  launch_apply_f64(p->coef, nb, x, y, 4, s);
  HIPCHK(hipGetLastError());
  return PPE_OK;
}

ppe_status ppe_rhs_to_source(const ppe_problem* p, int32_t nb, const float* b, float* f, hipStream_t s) {
  if (!p || nb < 0 || (nb > 0 && (!b || !f))) return set_error(PPE_ERR_INVALID_ARG, "bad arguments");
  if (nb == 0) return PPE_OK;
  launch_rhs_to_source(p->coef, nb, b, f, s);
  HIPCHK(hipGetLastError());
  return PPE_OK;
}

ppe_status ppe_apply_precond(ppe_problem* p, int32_t nb, const float* r, float* z, const ppe_solve_opts* opts,
                             hipStream_t s) {
  ppe_solve_opts o;
  ppe_solve_opts_default(&o);
  if (opts) o = *opts;
  o.record_history = 0;
  ppe_status st = check_solve_args(p, nb, r, z, &o);
  if (st == PPE_OK) st = reject_solid(p, "ppe_apply_precond");
  if (st != PPE_OK) return st;
  if (nb == 0) return PPE_OK;
  const int64_t N = (int64_t)p->nx * p->ny * nb;
  if (o.precond == PPE_PC_NONE) {
    HIPCHK(hipMemcpyAsync(z, r, sizeof(float) * N, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return PPE_OK;
  }
  st = ensure_ws(p, nb);
  if (st != PPE_OK) return st;
  const int R = default_rows(p, nb);
  PcgArgs a = make_pcg_args(p, nb, R, o.precond == PPE_PC_JACOBI, o.tol, o.tol_kind, o.zero_x0);
  st = attach_extras(p, a, nb, o, s);
  if (st != PPE_OK) return st;
  a.r = const_cast<float*>(r);  // only read, as the PCG's residual
  launch_zero_flags(a.flags, nb, s);
  if (o.precond == PPE_PC_JACOBI) {
    launch_direction(a, nb, PPE_DIR_JACOBI, z, s);
  } else {
    if (o.precond == PPE_PC_MG) launch_vcycle(a, nb, s);
    else launch_ic(a, nb, s);
    HIPCHK(hipMemcpyAsync(z, a.z, sizeof(float) * N, hipMemcpyDeviceToDevice, s));
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return PPE_OK;
}

ppe_status ppe_solve_plain(ppe_problem* p, int32_t nb, const float* f, double* x,
                           const ppe_solve_opts* opts, ppe_solve_stats* stats, hipStream_t s) {
  ppe_solve_opts o;
  ppe_solve_opts_default(&o);
  if (opts) o = *opts;
  ppe_status st = check_solve_args(p, nb, f, x, &o);
  if (st != PPE_OK) return st;
  if (nb == 0) return PPE_OK;
  return solve_plain_impl(p, nb, f, x, o, stats, s);
}

ppe_status ppe_profile_pcg(ppe_problem* p, int32_t nb, const float* f, double* x,
                           const ppe_solve_opts* opts, int32_t reps, double* ms_out, hipStream_t s) {
  ppe_solve_opts o;
  ppe_solve_opts_default(&o);
  if (opts) o = *opts;
  ppe_status st = check_solve_args(p, nb, f, x, &o);
  if (st == PPE_OK) st = reject_solid(p, "ppe_profile_pcg");
  if (st != PPE_OK) return st;
  if (nb < 1 || reps < 1 || !ms_out) return set_error(PPE_ERR_INVALID_ARG, "nb, reps >= 1 and ms_out required");
  int form, R;
  resolve_plain(p, nb, o, &form, &R);
  return profile_form(p, nb, f, x, o, form, R, reps, ms_out, s);
}

ppe_status ppe_tune_pcg(ppe_problem* p, int32_t nb, const float* f, double* x, int32_t reps,
                        ppe_tune_result* out, hipStream_t s) {
  ppe_solve_opts o;
  ppe_solve_opts_default(&o);
  ppe_status st = check_solve_args(p, nb, f, x, &o);
  if (st == PPE_OK) st = reject_solid(p, "ppe_tune_pcg");
  if (st != PPE_OK) return st;
  if (nb < 1 || reps < 2) return set_error(PPE_ERR_INVALID_ARG, "nb >= 1 and reps >= 2 required");
  // Candidates run the real iteration on (f, x) without a stopping test.
  o.tol = 0.0;
  o.max_iter = 1 << 30;
  o.zero_x0 = 1;
  static const int kRows[6] = {2, 4, 8, 16, 20, 24};
  static const int kForms[3] = {PPE_PCG_SINGLE_REDUCTION, PPE_PCG_TWO_PHASE, PPE_PCG_TWO_STEP};
  ppe_tune_result res{};
  // The untuned default (two-step form, height from its cost model) is kept
  // unless another configuration is more than 3 % faster, so that timing
  // noise between near-equal candidates does not flip the choice.
  const int def_rows = default_rows_two_step(&p, 1, nb);
  double def_us = 0.0;
  for (int v = 0; v < 3; ++v)
    for (int k = 0; k < 6; ++k) {
      if (!height_ok(kForms[v], kRows[k])) continue;
      double ms[2] = {0, 0};
      st = profile_form(p, nb, f, x, o, kForms[v], kRows[k], reps, ms, s);
      if (st != PPE_OK) return st;
      const double us = (ms[0] + ms[1]) * 1e3 / (kForms[v] == PPE_PCG_TWO_STEP ? 2.0 : 1.0);
      res.us_per_iter[v][k] = us;
      if (kForms[v] == PPE_PCG_TWO_STEP && kRows[k] == def_rows) def_us = us;
    }
  double best = def_us;
  int bv = PPE_PCG_TWO_STEP, br = def_rows;
  for (int v = 0; v < 3; ++v)
    for (int k = 0; k < 6; ++k) {
      const double us = res.us_per_iter[v][k];
      if (us > 0.0 && us < 0.97 * def_us && us < best) {
        best = us;
        bv = kForms[v];
        br = kRows[k];
      }
    }
  res.variant = bv;
  res.rows_per_wave = br;
  st = ppe_set_tuning(p, nb, bv, br);
  if (st != PPE_OK) return st;
  if (out) *out = res;
  return PPE_OK;
}

ppe_status ppe_set_tuning(ppe_problem* p, int32_t nb, int32_t variant, int32_t rows_per_wave) {
  if (!p || nb < 1) return set_error(PPE_ERR_INVALID_ARG, "problem and nb >= 1 required");
  if (variant != PPE_PCG_SINGLE_REDUCTION && variant != PPE_PCG_TWO_PHASE && variant != PPE_PCG_TWO_STEP)
    return set_error(PPE_ERR_INVALID_ARG, "variant must be single-reduction, two-phase or two-step");
  if (!height_ok(variant, rows_per_wave))
    return set_error(PPE_ERR_INVALID_ARG, "rows_per_wave must be 2, 4, 8 or 16 (two-step: also 20 or 24)");
  for (auto& t : p->tuned)
    if (t[0] == nb) {
      t = {nb, variant, rows_per_wave};
      return PPE_OK;
    }
  p->tuned.push_back({nb, variant, rows_per_wave});
  return PPE_OK;
}

ppe_status ppe_get_tuning(const ppe_problem* p, int32_t nb, int32_t* variant, int32_t* rows_per_wave) {
  if (!p || nb < 1 || !variant || !rows_per_wave) return set_error(PPE_ERR_INVALID_ARG, "bad arguments");
  ppe_solve_opts o;
  ppe_solve_opts_default(&o);
  int form, R;
  resolve_plain(p, nb, o, &form, &R);
  *variant = form;
  *rows_per_wave = R;
  return PPE_OK;
}

ppe_status ppe_profile_copy(const void* src, void* dst, int64_t bytes, int32_t reps, double* ms_out,
                            hipStream_t s) {
  if (!src || !dst || bytes <= 0 || bytes % 16 || reps < 1 || !ms_out)
    return set_error(PPE_ERR_INVALID_ARG, "copy needs buffers, bytes > 0 divisible by 16, reps >= 1");
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  for (int k = 0; k < reps; ++k) launch_copy16(src, dst, bytes / 16, s);
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  float t = 0;
  HIPCHK(hipEventElapsedTime(&t, e0, e1));
  ms_out[0] = t / reps;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return PPE_OK;
}

}  // extern "C"
