// Hybrid solve of Sec. 2.2: rounds of Num_CG-type (Jacobi-)PCG iterations and
// Num_DLSM line-search steps along the network's error estimate (Eqs. 11-13),
// restarting PCG after each line-search block. One round is captured as a HIP
// graph and replayed until every solve of the batch has finished; each round
// ends with a reliable update (FP64 true residual), which is also where
// convergence is judged.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

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
  // phase clocks (device real-time clock): 0 CG-type, 1 network, 2 line search
  int par = 0;
  for (int r = 0; r < rounds; ++r) {
    for (int c = 0; c < o.num_cg; ++c) {
      launch_pcg_pair(a, nb, par, 0, 0, s);
      par ^= 1;
    }
    const int lastpar = par ^ 1;
    if (o.num_cg > 0) launch_hist_cg(a, nb, lastpar, s);
    launch_mark(a, nb, 0, s);
    for (int d = 0; d < o.num_dlsm; ++d) {
      if (o.direction == PPE_DIR_NET) {
        ppe_status st = net_forward(p, net, nb, a.r, const_cast<float*>(a.e), s);
        if (st != PPE_OK) return st;
      } else {
        launch_direction(a, nb, o.direction, const_cast<float*>(a.e), s);
      }
      launch_mark(a, nb, 1, s);
      launch_dlsm_step(a, nb, lastpar, s);
      launch_mark(a, nb, 2, s);
    }
    launch_pcg_pair(a, nb, par, 1, 1, s);  // reliable update + CG restart
    par ^= 1;
  }
  HIPCHK(hipGetLastError());
  return PPE_OK;
}

// One hybrid solve (of nb right-hand sides on one problem) in progress: its
// arguments and the graph of one replay unit.
struct HybridRun {
  ppe_problem* p = nullptr;
  int nb = 0;
  PcgArgs a{};
  hipGraphExec_t exec = nullptr;
  int per = 1;               // rounds per replay unit
  int64_t max_units = 0;
  bool done = false;         // every solve of the run has reached a decision
  bool pending = false;      // a unit's flags are in flight
};

// Setup of a run on stream s: workspace, network constants, call arguments,
// the first true residual, and the capture of one replay unit.
static ppe_status hybrid_begin(HybridRun& h, ppe_problem* p, ppe_net* net, int32_t nb, const float* f, double* x,
                               const ppe_solve_opts& o, hipStream_t s, bool capture = true) {
  h.p = p;
  h.nb = nb;
  ppe_status st = ensure_ws(p, nb);
  if (st != PPE_OK) return st;
  if (o.direction == PPE_DIR_NET) {
    st = net_cache_ensure(p, net, nb, s);
    if (st != PPE_OK) return st;
  }
  const int R = rows_of(p, nb, o);
  h.a = make_pcg_args(p, nb, R, o.precond == PPE_PC_JACOBI, o.tol, o.tol_kind, o.zero_x0);
  st = attach_extras(p, h.a, nb, o, s);
  if (st != PPE_OK) return st;
  // The reliable update closing every round replaces the delta trigger.
  launch_set_call(p->ws.call, f, x, o.max_iter, 0.0, s);
  launch_pcg_setup(h.a, nb, s);
  HIPCHK(hipGetLastError());
  // Rounds per replayed unit: the parity must return to 0 at its end.
  h.per = ((o.num_cg + 1) % 2) ? 2 : 1;
  if (o.use_graph && capture) {
    if (!p->cap_stream) HIPCHK(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    st = enqueue_rounds(p, net, h.a, nb, o, h.per, p->cap_stream);
    hipError_t e = hipStreamEndCapture(p->cap_stream, &graph);
    if (st != PPE_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return set_error(PPE_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&h.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      h.exec = nullptr;
      return set_error(PPE_ERR_HIP, "graph instantiate failed: %s", hipGetErrorString(e));
    }
  }
  const int iters_per_unit = h.per * (o.num_cg + o.num_dlsm);
  h.max_units = (int64_t)o.max_iter / (iters_per_unit > 0 ? iters_per_unit : 1) + 3;
  return PPE_OK;
}

// Enqueues unit c of a run, then the copy of its done flags to the host and
// an event behind them (double-buffered by the parity of c).
static ppe_status hybrid_unit(HybridRun& h, ppe_net* net, const ppe_solve_opts& o, int64_t c, hipStream_t s) {
  SolveWs& w = h.p->ws;
  if (h.exec) {
    HIPCHK(hipGraphLaunch(h.exec, s));
  } else {
    ppe_status st = enqueue_rounds(h.p, net, h.a, h.nb, o, h.per, s);
    if (st != PPE_OK) return st;
  }
  HIPCHK(hipMemcpyAsync(w.h_flags + (c & 1) * h.nb, w.flags, sizeof(int32_t) * h.nb, hipMemcpyDeviceToHost, s));
  HIPCHK(hipEventRecord(w.ev[c & 1], s));
  h.pending = true;
  return PPE_OK;
}

// Waits for the flags of unit c and records whether every solve has decided.
static ppe_status hybrid_check(HybridRun& h, int64_t c) {
  SolveWs& w = h.p->ws;
  HIPCHK(hipEventSynchronize(w.ev[c & 1]));
  const int32_t* fl = w.h_flags + (c & 1) * h.nb;
  bool all = true;
  for (int i = 0; i < h.nb; ++i) all = all && fl[i] != DONE_NO;
  h.done = all;
  return PPE_OK;
}

static void hybrid_release(HybridRun& h) {
  if (h.exec) (void)hipGraphExecDestroy(h.exec);
  h.exec = nullptr;
}

ppe_status solve_hybrid_impl(ppe_problem* p, ppe_net* net, int32_t nb, const float* f, double* x,
                             const ppe_solve_opts& o, ppe_solve_stats* stats, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  HybridRun h;
  ppe_status st = hybrid_begin(h, p, net, nb, f, x, o, s);
  if (st != PPE_OK) {
    hybrid_release(h);
    return st;
  }
  for (int64_t c = 0; c < h.max_units && st == PPE_OK; ++c) {
    st = hybrid_unit(h, net, o, c, s);
    if (st == PPE_OK && c >= 1) st = hybrid_check(h, c - 1);
    if (h.done) break;
  }
  hybrid_release(h);
  if (st != PPE_OK) return st;
  launch_pcg_finish(h.a, nb, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return fill_stats(p, nb, stats, ms, s, true, h.a);
}

// Statistics of every solve of a batch, and the batch status (the worst).
static ppe_status batch_stats(int32_t n, ppe_problem* const* problems, const std::vector<HybridRun>& runs,
                              ppe_solve_stats* stats, std::chrono::steady_clock::time_point t0, hipStream_t s) {
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  ppe_status worst = PPE_OK;
  for (int i = 0; i < n; ++i) {
    const ppe_status st = fill_stats(problems[i], 1, stats ? stats + i : nullptr, ms, s, true, runs[i].a);
    if (st == PPE_ERR_NONFINITE) worst = st;
    else if (st == PPE_NOT_CONVERGED && worst == PPE_OK) worst = st;
    else if (st < 0 && st != PPE_ERR_NONFINITE) return st;
  }
  if (worst == PPE_ERR_NONFINITE) set_error(worst, "non-finite value in a source field or iteration");
  return worst;
}

// Rounds of the runs `live` of a lock-step batch with the network direction:
// every run's launches in the order of enqueue_rounds, the forwards of all
// runs as one grouped launch per layer (members whose solve has decided
// return at once, as every other kernel of a decided solve does).
static ppe_status enqueue_rounds_group(const std::vector<HybridRun*>& live, const NetGroup& G,
                                       const ppe_solve_opts& o, int rounds, hipStream_t s) {
  int par = 0;
  for (int r = 0; r < rounds; ++r) {
    for (int c = 0; c < o.num_cg; ++c) {
      for (HybridRun* h : live) launch_pcg_pair(h->a, h->nb, par, 0, 0, s);
      par ^= 1;
    }
    const int lastpar = par ^ 1;
    for (HybridRun* h : live) {
      if (o.num_cg > 0) launch_hist_cg(h->a, h->nb, lastpar, s);
      launch_mark(h->a, h->nb, 0, s);
    }
    for (int d = 0; d < o.num_dlsm; ++d) {
      ppe_status st = net_group_forward(G, s);
      if (st != PPE_OK) return st;
      for (HybridRun* h : live) {
        launch_mark(h->a, h->nb, 1, s);
        launch_dlsm_step(h->a, h->nb, lastpar, s);
        launch_mark(h->a, h->nb, 2, s);
      }
    }
    for (HybridRun* h : live) launch_pcg_pair(h->a, h->nb, par, 1, 1, s);
    par ^= 1;
  }
  HIPCHK(hipGetLastError());
  return PPE_OK;
}

// Lock-step batch with the network direction: one replay unit for all runs
// that have not decided, rebuilt (group tables and graph) whenever at most
// half of the runs it was built for are left, so that decided solves cost
// launches of empty workgroups for at most a factor of two.
static ppe_status batch_group_loop(std::vector<HybridRun>& runs, ppe_net* net, const ppe_solve_opts& o,
                                   hipStream_t s, std::vector<NetGroup>& groups,
                                   std::vector<hipGraphExec_t>& execs) {
  std::vector<HybridRun*> live;
  for (HybridRun& h : runs) live.push_back(&h);
  size_t built_for = 0;
  hipGraphExec_t exec = nullptr;
  auto rebuild = [&]() -> ppe_status {
    std::vector<ppe_problem*> probs;
    std::vector<const float*> r;
    std::vector<float*> e;
    std::vector<const int32_t*> skip;
    for (HybridRun* h : live) {
      probs.push_back(h->p);
      r.push_back(h->a.r);
      e.push_back(const_cast<float*>(h->a.e));
      skip.push_back(h->a.flags);
    }
    groups.emplace_back();
    ppe_status st = net_group_build((int)live.size(), probs.data(), net, r.data(), e.data(), skip.data(), s,
                                    groups.back());
    if (st != PPE_OK) return st;
    built_for = live.size();
    exec = nullptr;
    if (!o.use_graph) return PPE_OK;
    ppe_problem* p0 = live[0]->p;
    if (!p0->cap_stream) HIPCHK(hipStreamCreateWithFlags(&p0->cap_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(p0->cap_stream, hipStreamCaptureModeThreadLocal));
    st = enqueue_rounds_group(live, groups.back(), o, live[0]->per, p0->cap_stream);
    hipError_t err = hipStreamEndCapture(p0->cap_stream, &graph);
    if (st != PPE_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (err != hipSuccess) return set_error(PPE_ERR_HIP, "graph capture failed: %s", hipGetErrorString(err));
    err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (err != hipSuccess) {
      exec = nullptr;
      return set_error(PPE_ERR_HIP, "graph instantiate failed: %s", hipGetErrorString(err));
    }
    execs.push_back(exec);
    return PPE_OK;
  };
  ppe_status st = rebuild();
  const int64_t max_units = runs[0].max_units;
  std::vector<HybridRun*> prev;  // the runs of the unit before
  for (int64_t c = 0; c < max_units && st == PPE_OK; ++c) {
    if (exec) {
      HIPCHK(hipGraphLaunch(exec, s));
    } else {
      st = enqueue_rounds_group(live, groups.back(), o, live[0]->per, s);
      if (st != PPE_OK) break;
    }
    for (HybridRun* h : live) {
      SolveWs& w = h->p->ws;
      HIPCHK(hipMemcpyAsync(w.h_flags + (c & 1) * h->nb, w.flags, sizeof(int32_t) * h->nb, hipMemcpyDeviceToHost, s));
      HIPCHK(hipEventRecord(w.ev[c & 1], s));
    }
    for (HybridRun* h : prev)
      if (!h->done && st == PPE_OK) st = hybrid_check(*h, c - 1);
    prev = live;
    std::vector<HybridRun*> next;
    for (HybridRun* h : live)
      if (!h->done) next.push_back(h);
    if (next.empty()) break;
    if (next.size() != live.size()) {
      live = next;
      if (2 * live.size() <= built_for && st == PPE_OK) st = rebuild();
    }
  }
  return st;
}

// Hybrid solves of a mixed-size batch: one run per problem, advanced in lock
// step on one stream. Each unit of a round enqueues the next replay of every
// run that has not yet decided, so the runs' rounds interleave; a run leaves
// the rotation once its flags show that its solve has decided.
ppe_status solve_hybrid_batch_impl(int32_t n, ppe_problem* const* problems, ppe_net* net, const float* const* f,
                                   double* const* x, const ppe_solve_opts& o, ppe_solve_stats* stats,
                                   hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<HybridRun> runs(n);
  ppe_status st = PPE_OK;
  const bool grouped = o.direction == PPE_DIR_NET;
  for (int i = 0; i < n && st == PPE_OK; ++i)
    st = hybrid_begin(runs[i], problems[i], net, 1, f[i], x[i], o, s, !grouped);
  if (grouped) {
    std::vector<NetGroup> groups;
    std::vector<hipGraphExec_t> execs;
    if (st == PPE_OK) st = batch_group_loop(runs, net, o, s, groups, execs);
    if (st == PPE_OK)
      for (const HybridRun& h : runs) launch_pcg_finish(h.a, 1, s);
    // the tables and graphs are in use until the stream has drained
    const hipError_t e = hipStreamSynchronize(s);
    for (hipGraphExec_t x : execs) (void)hipGraphExecDestroy(x);
    for (NetGroup& g : groups) net_group_free(g);
    for (HybridRun& h : runs) hybrid_release(h);
    if (st != PPE_OK) return st;
    if (e != hipSuccess) return set_error(PPE_ERR_HIP, "hipStreamSynchronize failed: %s", hipGetErrorString(e));
    return batch_stats(n, problems, runs, stats, t0, s);
  }
  int64_t max_units = 0;
  for (const HybridRun& h : runs) max_units = std::max(max_units, h.max_units);
  for (int64_t c = 0; c < max_units && st == PPE_OK; ++c) {
    bool any = false;
    for (HybridRun& h : runs) {
      if (h.done || c >= h.max_units) continue;
      st = hybrid_unit(h, net, o, c, s);
      if (st != PPE_OK) break;
      any = true;
    }
    if (st != PPE_OK || !any) break;
    if (c >= 1)
      for (HybridRun& h : runs)
        if (!h.done && c - 1 < h.max_units && st == PPE_OK) st = hybrid_check(h, c - 1);
  }
  for (HybridRun& h : runs) hybrid_release(h);
  if (st != PPE_OK) return st;
  for (const HybridRun& h : runs) launch_pcg_finish(h.a, 1, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return batch_stats(n, problems, runs, stats, t0, s);
}

}  // namespace ppe

using namespace ppe;

extern "C" ppe_status ppe_solve_hybrid(ppe_problem* p, ppe_net* net, int32_t nb, const float* f, double* x,
                                       const ppe_solve_opts* opts, ppe_solve_stats* stats, hipStream_t s) {
  ppe_solve_opts o;
  ppe_solve_opts_default(&o);
  if (opts) o = *opts;
  ppe_status st = check_solve_args(p, nb, f, x, &o);
  if (st == PPE_OK) st = reject_solid(p, "ppe_solve_hybrid");
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
