// Allocation-free plain solve: the PCG of ppe_solve_plain for one right-hand
// side, run in a fixed device array of this translation unit instead of the
// problem's workspace, with eager launches and synchronous polling (no HIP
// graph, event, pinned buffer or device allocation). Its kernels are those of
// ppe_solve_plain; only where the vectors, partial sums and state live
// differs, so a call gives the same bits as ppe_solve_plain with the same
// iteration form and tile height.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <mutex>

#include "api_internal.hpp"

namespace ppe {

// The scratch array. In host code `scratch` names a host-side stand-in, not
// device memory: every host use goes through the device address that
// hipGetSymbolAddress returns for the current device (scratch_base below).
static __device__ __align__(256) unsigned char scratch[PPE_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;                       // serialises calls (one scratch array per device)
void* g_base[kMaxDevices] = {nullptr};  // device address of `scratch`, per device

// Device address of the current device's scratch array, looked up once per
// device with that device current.
ppe_status scratch_base(unsigned char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(PPE_ERR_HIP, "hipGetDevice failed: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return set_error(PPE_ERR_HIP, "device index %d out of range", dev);
  if (!g_base[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return set_error(PPE_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_base[dev] = ptr;
  }
  *out = (unsigned char*)g_base[dev];
  return PPE_OK;
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// Byte layout of one solve in the scratch array: vectors, partial sums,
// state, flag, call arguments.
struct Layout {
  size_t vec, part, st, flags, call, total;
  int Pmax, P2max;
};

Layout layout_of(const ppe_problem* p) {
  Layout L{};
  ws_extent(p, &L.Pmax, &L.P2max);
  const size_t N = (size_t)p->nx * p->ny;
  size_t o = 0;
  L.vec = o;
  o += round256(sizeof(float) * 6 * N);
  L.part = o;
  o += round256(sizeof(double) * (16 * (size_t)L.Pmax + 22 * (size_t)L.P2max));
  L.st = o;
  o += round256(sizeof(SolveState));
  L.flags = o;
  o += round256(sizeof(int32_t));
  L.call = o;
  o += round256(sizeof(CallArgs));
  L.total = o;
  return L;
}

// Zero fill of n 32-bit words (graph-safe, unlike a memset node).
__global__ void k_zero_words(uint32_t* p, int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    p[k] = 0u;
}

void zero_words(void* p, size_t bytes, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 4);
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
  k_zero_words<<<blocks > 0 ? blocks : 1, 256, 0, s>>>((uint32_t*)p, n);
}

}  // namespace
}  // namespace ppe

using namespace ppe;

#define HIPCHK(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return set_error(PPE_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

extern "C" int64_t ppe_noalloc_scratch_bytes(const ppe_problem* p) {
  if (!p) return -1;
  return (int64_t)layout_of(p).total;
}

extern "C" ppe_status ppe_solve_plain_noalloc(const ppe_problem* p, const float* f, double* x,
                                              const ppe_solve_opts* opts, ppe_solve_stats* stats, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  ppe_solve_opts o;
  ppe_solve_opts_default(&o);
  if (opts) o = *opts;
  ppe_status st = check_solve_args(p, 1, f, x, &o);
  if (st != PPE_OK) return st;
  if (o.precond == PPE_PC_MG || o.precond == PPE_PC_IC || o.record_history || p->mask_mode == PPE_MASK_SOLID)
    return set_error(PPE_ERR_UNSUPPORTED,
                     "the allocation-free solve runs Jacobi or no preconditioning on unmasked operators, "
                     "without history");
  const Layout L = layout_of(p);
  if (L.total > (size_t)PPE_NOALLOC_SCRATCH_BYTES)
    return set_error(PPE_ERR_INVALID_ARG,
                     "a %d x %d grid needs %zu bytes of solver state; the allocation-free solve holds %zu "
                     "(use ppe_solve_plain)",
                     p->nx, p->ny, L.total, (size_t)PPE_NOALLOC_SCRATCH_BYTES);
  std::lock_guard<std::mutex> lock(g_mu);
  unsigned char* base = nullptr;
  st = scratch_base(&base);
  if (st != PPE_OK) return st;
  int form, R;
  resolve_plain(p, 1, o, &form, &R);
  const WsView v{(float*)(base + L.vec), (double*)(base + L.part), L.Pmax, (SolveState*)(base + L.st),
                 (int32_t*)(base + L.flags), (CallArgs*)(base + L.call)};
  const PcgArgs a = make_pcg_args_at(p, v, 1, R, o.precond == PPE_PC_JACOBI, o.tol, o.tol_kind, o.zero_x0);
  // The array keeps the previous call's contents: clear the partial sums,
  // the state, the flag and the call arguments before the set-up.
  zero_words(base + L.part, L.total - L.part, s);
  launch_set_call(v.call, f, x, o.max_iter, o.reliable_delta * o.reliable_delta, s);
  launch_setup(a, 1, form, s);
  HIPCHK(hipGetLastError());
  int chunk = o.chunk > 0 ? o.chunk : 64;
  chunk += chunk & 1;
  const int64_t max_chunks = (3 * (int64_t)o.max_iter + 8) / chunk + 2;
  for (int64_t c = 0; c < max_chunks; ++c) {
    launch_chunk(a, 1, chunk, form, s);
    HIPCHK(hipGetLastError());
    int32_t flag = DONE_NO;
    HIPCHK(hipMemcpyAsync(&flag, v.flags, sizeof flag, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (flag != DONE_NO) break;
  }
  launch_pcg_finish(a, 1, s);
  HIPCHK(hipGetLastError());
  SolveState S;
  HIPCHK(hipMemcpyAsync(&S, v.st, sizeof S, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  st = state_status(S);
  if (stats) {
    double* hbuf = stats->history;
    const int hcap = stats->history_cap;
    stats_from_state(S, st, ms, false, stats);
    stats->ms_pcg = stats->ms_device;
    stats->history = hbuf;
    stats->history_cap = hcap;
  }
  if (st == PPE_ERR_NONFINITE) set_error(st, "non-finite value in the source field or iteration");
  return st;
}
