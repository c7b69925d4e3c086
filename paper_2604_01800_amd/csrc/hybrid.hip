// Hybrid solve of Sec. 2.2: rounds of Num_CG-type (Jacobi-)PCG iterations and
// Num_DLSM line-search steps along the network's error estimate (Eqs. 11-13),
// restarting PCG after each line-search block. One round is captured as a HIP
// graph and replayed until every solve of the batch has finished; each round
// ends with a reliable update (FP64 true residual), which is also where
// convergence is judged.
#include <hip/hip_runtime.h>

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

// Enqueues `rounds` hybrid rounds starting at parity 0 on stream s.
static ppe_status enqueue_rounds(ppe_problem* p, ppe_net* net, const PcgArgs& a, int nb, const ppe_solve_opts& o,
                                 int rounds, hipStream_t s) {
  int par = 0;
  for (int r = 0; r < rounds; ++r) {
    for (int c = 0; c < o.num_cg; ++c) {
      launch_pcg_pair(a, nb, par, 0, 0, s);
      par ^= 1;
    }
    const int lastpar = par ^ 1;
    for (int d = 0; d < o.num_dlsm; ++d) {
      if (o.direction == PPE_DIR_NET) {
        ppe_status st = net_forward(p, net, nb, a.r, const_cast<float*>(a.e), s);
        if (st != PPE_OK) return st;
      } else {
        launch_direction(a, nb, o.direction, const_cast<float*>(a.e), s);
      }
      launch_dlsm_step(a, nb, lastpar, s);
    }
    launch_pcg_pair(a, nb, par, 1, 1, s);  // reliable update + CG restart
    par ^= 1;
  }
  HIPCHK(hipGetLastError());
  return PPE_OK;
}

ppe_status solve_hybrid_impl(ppe_problem* p, ppe_net* net, int32_t nb, const float* f, double* x,
                             const ppe_solve_opts& o, ppe_solve_stats* stats, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  ppe_status st = ensure_ws(p, nb);
  if (st != PPE_OK) return st;
  if (o.direction == PPE_DIR_NET) {
    st = net_cache_ensure(p, net, nb, s);
    if (st != PPE_OK) return st;
  }
  const int R = rows_of(p, nb, o);
  const PcgArgs a = make_pcg_args(p, nb, R, o.precond == PPE_PC_JACOBI, o.tol, o.tol_kind, o.zero_x0);
  // The reliable update closing every round replaces the delta trigger.
  launch_set_call(p->ws.call, f, x, o.max_iter, 0.0, s);
  launch_pcg_setup(a, nb, s);
  HIPCHK(hipGetLastError());
  // Rounds per replayed unit: the parity must return to 0 at its end.
  const int per = ((o.num_cg + 1) % 2) ? 2 : 1;
  SolveWs& w = p->ws;
  hipGraphExec_t exec = nullptr;
  if (o.use_graph) {
    if (!p->cap_stream) HIPCHK(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    st = enqueue_rounds(p, net, a, nb, o, per, p->cap_stream);
    hipError_t e = hipStreamEndCapture(p->cap_stream, &graph);
    if (st != PPE_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return set_error(PPE_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return set_error(PPE_ERR_HIP, "graph instantiate failed: %s", hipGetErrorString(e));
  }
  const int iters_per_unit = per * (o.num_cg + o.num_dlsm);
  const int64_t max_units = (int64_t)o.max_iter / (iters_per_unit > 0 ? iters_per_unit : 1) + 3;
  for (int64_t c = 0; c < max_units; ++c) {
    if (exec) {
      HIPCHK(hipGraphLaunch(exec, s));
    } else {
      st = enqueue_rounds(p, net, a, nb, o, per, s);
      if (st != PPE_OK) return st;
    }
    HIPCHK(hipMemcpyAsync(w.h_flags + (c & 1) * nb, w.flags, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(w.ev[c & 1], s));
    if (c >= 1) {
      HIPCHK(hipEventSynchronize(w.ev[(c - 1) & 1]));
      const int32_t* fl = w.h_flags + ((c - 1) & 1) * nb;
      bool all = true;
      for (int i = 0; i < nb; ++i) all = all && fl[i] != DONE_NO;
      if (all) break;
    }
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  launch_pcg_finish(a, nb, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return fill_stats(p, nb, stats, ms, s, true);
}

}  // namespace ppe

using namespace ppe;

extern "C" ppe_status ppe_solve_hybrid(ppe_problem* p, ppe_net* net, int32_t nb, const float* f, double* x,
                                       const ppe_solve_opts* opts, ppe_solve_stats* stats, hipStream_t s) {
  ppe_solve_opts o;
  ppe_solve_opts_default(&o);
  if (opts) o = *opts;
  ppe_status st = check_solve_args(p, nb, f, x, &o);
  if (st != PPE_OK) return st;
  if (o.num_cg < 0 || o.num_dlsm < 0 || o.num_cg + o.num_dlsm < 1 || o.num_cg > 64 || o.num_dlsm > 64)
    return set_error(PPE_ERR_INVALID_ARG, "num_cg, num_dlsm must lie in [0, 64] with a positive sum");
  if (o.direction < PPE_DIR_NET || o.direction > PPE_DIR_ONES)
    return set_error(PPE_ERR_INVALID_ARG, "unknown direction %d", o.direction);
  if (o.direction == PPE_DIR_NET) {
    if (!net) return set_error(PPE_ERR_INVALID_ARG, "net is NULL");
    st = check_net_grid(p, net);
    if (st != PPE_OK) return st;
  }
  if (nb == 0) return PPE_OK;
  return solve_hybrid_impl(p, net, nb, f, x, o, stats, s);
}
