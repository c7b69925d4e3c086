// Host-side internals shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <string>
#include <vector>

#include "../../include/ppe.h"
#include "kernels.hpp"

namespace ppe {

// Solver workspace of one problem (grown on demand to the largest batch).
struct SolveWs {
  int nb = 0;
  int Pmax = 0;
  int P2max = 0;
  float* vec = nullptr;      // x_c, r, p0, p1, e, r1: [6][nb][N]
  double* part = nullptr;    // partial sums: [16][nb][Pmax], then [22][nb][P2max]
  SolveState* st = nullptr;  // [nb]
  int32_t* flags = nullptr;  // [nb]
  CallArgs* call = nullptr;
  int32_t* h_flags = nullptr;     // pinned [2][nb]
  SolveState* h_state = nullptr;  // pinned [nb]
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipGraphExec_t exec = nullptr;
  std::array<int64_t, 8> exec_key{};  // launch configuration the graph was captured for
  double* hist = nullptr;             // [nb][hist_cap] residual histories
  int64_t hist_elems = 0;
};

// Device workspace of the training-data generator (grown on demand).
struct GenWs {
  int nb = 0, J = 0, P = 0;
  int64_t N = 0;
  void* feat = nullptr;     // [nb][J] double4 (w_x, w_y, phi, l)
  double* raw = nullptr;    // [nb][N]
  double* part = nullptr;   // [nb][2][P]
  Coef* coefs = nullptr;    // [nb]
};

struct NetCache;  // per (grid, net) constants of the network (net_internal.hpp)
void net_cache_free(NetCache* c);
struct MgData;    // multigrid hierarchy of a problem (mg_internal.hpp)
void mg_free(MgData* m);

}  // namespace ppe

struct ppe_problem {
  int nx = 0, ny = 0;
  // Identity of this handle for caches keyed on problems: unique over the
  // process lifetime, unlike the handle's address, which the allocator reuses
  // after ppe_problem_destroy.
  uint64_t uid = 0;
  // Tuned PCG launch configuration per batch size: {nb, variant, rows_per_wave}.
  std::vector<std::array<int, 3>> tuned;
  std::vector<double> xc, yc, hx, hy;
  std::vector<uint8_t> mask;  // empty = no obstacle
  int mask_mode = PPE_MASK_DIBPM;
  // device copies of the 1D coefficients
  void* dev_coef = nullptr;
  uint8_t* d_mask = nullptr;
  float* d_solid = nullptr;  // solid-mask mode: fluid flags, then the inverse diagonal
  ppe::Coef coef{};
  ppe::SolveWs ws;
  hipStream_t cap_stream = nullptr;
  ppe::NetCache* net_cache = nullptr;
  ppe::MgData* mg = nullptr;
  // incomplete-Cholesky preconditioner: 1/D on red cells, 1/S on black cells,
  // and its output z for up to ic_nb right-hand sides
  float* d_icq = nullptr;
  float* d_icz = nullptr;
  int ic_nb = 0;
};

namespace ppe {
extern thread_local std::string g_last_error;
ppe_status set_error(ppe_status st, const char* fmt, ...);
void* dev_alloc(size_t bytes);
void dev_free(void* p);
ppe_status problem_upload(ppe_problem* p, hipStream_t s);
ppe_status coef_upload(int nx, int ny, const double* hx, const double* hy, const double* gx, const double* gy,
                       const double* xc, const double* yc, hipStream_t s, std::vector<double>& h64,
                       std::vector<float>& h32, void** dev, Coef* cout);
void problem_release(ppe_problem* p);
ppe_status ensure_ws(ppe_problem* p, int nb);
// Device buffers a solve of nb systems runs in: the problem's own workspace
// (make_pcg_args) or a caller's view of equal layout (make_pcg_args_at).
struct WsView {
  float* vec;        // [6][nb][N]
  double* part;      // [16][nb][Pmax], then [22][nb][P2max]
  int Pmax;
  SolveState* st;    // [nb]
  int32_t* flags;    // [nb]
  CallArgs* call;
};
// Workgroup counts the partial-sum arrays of a problem are sized for.
void ws_extent(const ppe_problem* p, int* Pmax, int* P2max);
PcgArgs make_pcg_args_at(const ppe_problem* p, const WsView& w, int nb, int R, int jacobi, double tol, int tol_kind,
                         int zero_x0);
PcgArgs make_pcg_args(ppe_problem* p, int nb, int R, int jacobi, double tol, int tol_kind, int zero_x0);
void launch_setup(const PcgArgs& a, int nb, int form, hipStream_t s);
void launch_chunk(const PcgArgs& a, int nb, int chunk, int form, hipStream_t s);
void stats_from_state(const SolveState& S, ppe_status st, double ms, bool hybrid, ppe_solve_stats* out);
ppe_status state_status(const SolveState& S);
int rows_of(const ppe_problem* p, int nb, const ppe_solve_opts& o);
ppe_status run_pcg_chunks(ppe_problem* p, const PcgArgs& a, int nb, const ppe_solve_opts& o, hipStream_t s,
                          int form);
// Resolves PPE_PCG_AUTO and rows_per_wave = 0 for a plain solve of nb systems:
// the tuned entry for nb if there is one, else the size heuristic.
ppe_status gen_ensure(GenWs& w, int nb, int64_t N, int J, int P);
void gen_free(GenWs& w);
ppe_status check_gen_opts(const ppe_train_opts& o);
// R [nb][N] FP32 for the batch of grids probs (one size), from opts' seed,
// step, length-scale range and feature count; synchronises stream s.
ppe_status generate_rhs(GenWs& w, int nb, ppe_problem* const* probs, const ppe_train_opts& o, float* R,
                        hipStream_t s);
double wall_clock_khz();
bool height_ok(int form, int R);
int default_rows_two_step(const ppe_problem* const* probs, int n, int nb);
void resolve_plain(const ppe_problem* p, int nb, const ppe_solve_opts& o, int* form, int* rows);
ppe_status profile_form(ppe_problem* p, int nb, const float* f, double* x, const ppe_solve_opts& o, int form,
                        int R, int reps, double* ms_out, hipStream_t s);
// Host statistics of the nb solves of a call (and the residual histories a
// recorded, into the callers' buffers).
ppe_status fill_stats(ppe_problem* p, int nb, ppe_solve_stats* stats, double ms, hipStream_t s, bool hybrid,
                      const PcgArgs& a);
// Attaches to a what the options ask for beyond the plain iteration: the
// multigrid hierarchy (PPE_PC_MG) and the device residual-history buffer.
ppe_status attach_extras(ppe_problem* p, PcgArgs& a, int nb, const ppe_solve_opts& o, hipStream_t s);
ppe_status check_solve_args(const ppe_problem* p, int32_t nb, const void* f, const void* x,
                            const ppe_solve_opts* opts);
// PPE_ERR_UNSUPPORTED for a solid-mask problem (entry points whose kernels
// carry only the immersed-boundary operator).
ppe_status reject_solid(const ppe_problem* p, const char* what);
}  // namespace ppe
