// Plain solves on grids of different sizes in one batch: every launch of the
// two-step kernel (two iterations) or of the single-reduction kernel (one
// iteration) runs over a work list of (solve, workgroup) entries, so small
// grids ride along with large ones instead of leaving the GPU idle. Each solve keeps its own workspace, scalars, partial
// sums and done flag; converged solves' workgroups exit at once. Chunks of
// iterations are captured as one HIP graph and replayed until every flag is
// set; the device records each solve's finishing time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>

#include "api_internal.hpp"
#include "net_internal.hpp"

namespace ppe {

#define HIPCHK(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return set_error(PPE_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

struct BatchWs {
  std::vector<uint64_t> key;  // uids of the problems the work list was built for
  int form = 0, R = 0, chunk = 0, jacobi = -1, n = 0, nblocks = 0;
  PcgArgs* d_descs = nullptr;
  uint32_t* d_work = nullptr;
  int32_t* d_flags = nullptr;
  int32_t* h_flags = nullptr;  // pinned [2][n]
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
};

static void batch_free(BatchWs& w) {
  if (w.exec) (void)hipGraphExecDestroy(w.exec);
  dev_free(w.d_descs);
  dev_free(w.d_work);
  dev_free(w.d_flags);
  if (w.h_flags) (void)hipHostFree(w.h_flags);
  for (auto& e : w.ev)
    if (e) (void)hipEventDestroy(e);
  if (w.cap) (void)hipStreamDestroy(w.cap);
  w = BatchWs{};
}

// (Re)builds the work list and buffers when the problem list, the form or
// the tile height changes.
static ppe_status batch_prepare(BatchWs& w, int n, ppe_problem* const* probs, int form, int R) {
  std::vector<uint64_t> key(n);
  for (int i = 0; i < n; ++i) key[i] = probs[i]->uid;
  if (w.d_descs && w.key == key && w.form == form && w.R == R) return PPE_OK;
  batch_free(w);
  std::vector<uint32_t> work;
  for (int i = 0; i < n; ++i) {
    // a multiple of 8, so that each solve's workgroups keep their XCD banding
    const uint32_t P = (form == PPE_PCG_TWO_STEP ? stencil_grid2(probs[i]->coef, R, 1) : stencil_grid(probs[i]->coef, R, 1)).x;
    if (P >= (1u << 20)) return set_error(PPE_ERR_SHAPE, "grid %d has too many tiles for a batch", i);
    for (uint32_t b = 0; b < P; ++b) work.push_back(((uint32_t)i << 20) | b);
  }
  w.d_descs = (PcgArgs*)dev_alloc(sizeof(PcgArgs) * n);
  w.d_work = (uint32_t*)dev_alloc(sizeof(uint32_t) * work.size());
  w.d_flags = (int32_t*)dev_alloc(sizeof(int32_t) * n);
  if (!w.d_descs || !w.d_work || !w.d_flags) {
    batch_free(w);
    return set_error(PPE_ERR_HIP, "allocation of the batch work list failed");
  }
  if (hipHostMalloc((void**)&w.h_flags, sizeof(int32_t) * 2 * n, hipHostMallocDefault) != hipSuccess) {
    batch_free(w);
    return set_error(PPE_ERR_HIP, "pinned host allocation failed");
  }
  for (auto& e : w.ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  HIPCHK(hipStreamCreateWithFlags(&w.cap, hipStreamNonBlocking));
  HIPCHK(hipMemcpy(w.d_work, work.data(), sizeof(uint32_t) * work.size(), hipMemcpyHostToDevice));
  w.key = key;
  w.form = form;
  w.R = R;
  w.n = n;
  w.nblocks = (int)work.size();
  return PPE_OK;
}

static void launch_batch_step(const BatchWs& w, bool jacobi, int par, hipStream_t s) {
  if (w.form == PPE_PCG_TWO_STEP) launch_pcg2_multi_step(w.d_descs, w.d_work, w.nblocks, w.R, jacobi, par, s);
  else launch_pcg1_multi_step(w.d_descs, w.d_work, w.nblocks, w.R, jacobi, par, s);
}

static void launch_batch_chunk(const BatchWs& w, bool jacobi, int chunk, hipStream_t s) {
  for (int k = 0; k < chunk; ++k) launch_batch_step(w, jacobi, k & 1, s);
}

static ppe_status batch_graph(BatchWs& w, bool jacobi, int chunk) {
  // The work list, form and height are fixed per BatchWs build (the graph is
  // destroyed with it), so chunk and preconditioner complete the key.
  if (w.exec && w.chunk == chunk && w.jacobi == (int)jacobi) return PPE_OK;
  if (w.exec) {
    (void)hipGraphExecDestroy(w.exec);
    w.exec = nullptr;
  }
  hipGraph_t graph = nullptr;
  HIPCHK(hipStreamBeginCapture(w.cap, hipStreamCaptureModeThreadLocal));
  launch_batch_chunk(w, jacobi, chunk, w.cap);
  hipError_t e = hipStreamEndCapture(w.cap, &graph);
  if (e != hipSuccess) return set_error(PPE_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&w.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    w.exec = nullptr;
    return set_error(PPE_ERR_HIP, "graph instantiate failed: %s", hipGetErrorString(e));
  }
  w.chunk = chunk;
  w.jacobi = jacobi;
  return PPE_OK;
}

}  // namespace ppe

using namespace ppe;

extern "C" ppe_status ppe_solve_batch(int32_t n, ppe_problem* const* problems, const ppe_net* net,
                                      const float* const* f, double* const* x, const ppe_solve_opts* opts,
                                      ppe_solve_stats* stats, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  if (n < 0) return set_error(PPE_ERR_INVALID_ARG, "n < 0");
  if (n == 0) return PPE_OK;
  if (n > 4096) return set_error(PPE_ERR_INVALID_ARG, "n > 4096");
  if (!problems || !f || !x) return set_error(PPE_ERR_INVALID_ARG, "problems, f or x is NULL");
  ppe_solve_opts o;
  ppe_solve_opts_default(&o);
  if (opts) o = *opts;
  int64_t cells = 0;
  for (int i = 0; i < n; ++i) {
    ppe_status st = check_solve_args(problems[i], 1, f[i], x[i], &o);
    if (st != PPE_OK) {
      const std::string msg = ppe_last_error();
      return set_error(st, "solve %d: %s", i, msg.c_str());
    }
    for (int k = 0; k < i; ++k)
      if (problems[k] == problems[i]) return set_error(PPE_ERR_INVALID_ARG, "problem %d appears twice", i);
    cells += (int64_t)problems[i]->nx * problems[i]->ny;
  }
  if (net) {
    // hybrid rounds (the two-phase CG form, as in ppe_solve_hybrid)
    if (o.num_cg < 0 || o.num_dlsm < 0 || o.num_cg + o.num_dlsm < 1 || o.num_cg > 64 || o.num_dlsm > 64)
      return set_error(PPE_ERR_INVALID_ARG, "num_cg, num_dlsm must lie in [0, 64] with a positive sum");
    if (o.direction < PPE_DIR_NET || o.direction > PPE_DIR_ONES)
      return set_error(PPE_ERR_INVALID_ARG, "unknown direction %d", o.direction);
    if (o.direction == PPE_DIR_NET)
      for (int i = 0; i < n; ++i) {
        ppe_status st = check_net_grid(problems[i], net);
        if (st != PPE_OK) {
          const std::string msg = ppe_last_error();
          return set_error(st, "solve %d: %s", i, msg.c_str());
        }
      }
    // the forward reads the network's parameters and writes only per-problem buffers
    return solve_hybrid_batch_impl(n, problems, const_cast<ppe_net*>(net), f, x, o, stats, s);
  }
  if (o.variant == PPE_PCG_TWO_PHASE)
    return set_error(PPE_ERR_UNSUPPORTED, "the mixed-size batch runs the two-step or single-reduction form");
  if (o.precond == PPE_PC_MG || o.precond == PPE_PC_IC || o.record_history)
    return set_error(PPE_ERR_UNSUPPORTED, "the plain mixed-size batch runs Jacobi or no preconditioning, without history");
  for (int i = 0; i < n; ++i)
    if (problems[i]->mask_mode == PPE_MASK_SOLID)
      return set_error(PPE_ERR_UNSUPPORTED, "the plain mixed-size batch does not take PPE_MASK_SOLID grids");
  const int form = o.variant == PPE_PCG_SINGLE_REDUCTION ? PPE_PCG_SINGLE_REDUCTION : PPE_PCG_TWO_STEP;
  int R = o.rows_per_wave;
  if (!height_ok(form, R))
    R = form == PPE_PCG_TWO_STEP ? default_rows_two_step(problems, n, 1)
        : (cells >= ((int64_t)1 << 20) ? 8 : cells >= ((int64_t)1 << 17) ? 4 : 2);
  const bool jacobi = o.precond == PPE_PC_JACOBI;
  static thread_local BatchWs w;
  ppe_status st = batch_prepare(w, n, problems, form, R);
  if (st != PPE_OK) return st;
  std::vector<PcgArgs> descs(n);
  for (int i = 0; i < n; ++i) {
    st = ensure_ws(problems[i], 1);
    if (st != PPE_OK) return st;
    descs[i] = make_pcg_args(problems[i], 1, R, jacobi, o.tol, o.tol_kind, o.zero_x0);
    descs[i].flags = w.d_flags + i;
  }
  HIPCHK(hipMemcpyAsync(w.d_descs, descs.data(), sizeof(PcgArgs) * n, hipMemcpyHostToDevice, s));
  for (int i = 0; i < n; ++i) {
    launch_set_call(problems[i]->ws.call, f[i], x[i], o.max_iter, o.reliable_delta * o.reliable_delta, s);
    launch_rhs(descs[i], 1, s);
    launch_pcg1_init(descs[i], 1, s);
  }
  launch_batch_step(w, jacobi, 1, s);  // true residual of x0
  HIPCHK(hipGetLastError());
  int chunk = o.chunk > 0 ? o.chunk : 64;
  chunk += chunk & 1;
  if (o.use_graph) {
    st = batch_graph(w, jacobi, chunk);
    if (st != PPE_OK) return st;
  }
  const int64_t max_chunks = (3 * (int64_t)o.max_iter + 8) / chunk + 2;
  for (int64_t c = 0; c < max_chunks; ++c) {
    if (o.use_graph) {
      HIPCHK(hipGraphLaunch(w.exec, s));
    } else {
      launch_batch_chunk(w, jacobi, chunk, s);
      HIPCHK(hipGetLastError());
    }
    HIPCHK(hipMemcpyAsync(w.h_flags + (c & 1) * n, w.d_flags, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(w.ev[c & 1], s));
    if (c >= 1) {
      HIPCHK(hipEventSynchronize(w.ev[(c - 1) & 1]));
      const int32_t* fl = w.h_flags + ((c - 1) & 1) * n;
      bool all = true;
      for (int i = 0; i < n; ++i) all = all && fl[i] != DONE_NO;
      if (all) break;
    }
  }
  for (int i = 0; i < n; ++i) launch_pcg_finish(descs[i], 1, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  ppe_status worst = PPE_OK;
  for (int i = 0; i < n; ++i) {
    st = fill_stats(problems[i], 1, stats ? stats + i : nullptr, ms, s, false, descs[i]);
    if (st == PPE_ERR_NONFINITE) worst = st;
    else if (st == PPE_NOT_CONVERGED && worst == PPE_OK) worst = st;
    else if (st < 0 && st != PPE_ERR_NONFINITE) return st;
  }
  if (worst == PPE_ERR_NONFINITE) set_error(worst, "non-finite value in a source field or iteration");
  return worst;
}
