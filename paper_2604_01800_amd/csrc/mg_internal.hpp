// Multigrid preconditioner of the PCG solve (the MGPCG CG-type of Sec. 2.5):
// device hierarchy and launchers shared by its host and kernel units.
#pragma once
#include <vector>

#include "api_internal.hpp"

namespace ppe {

// Chebyshev smoother on D^-1 A over [kChebLo, kChebHi] (kChebHi bounds the
// spectrum of D^-1 A: zero row sums and non-positive off-diagonals), degree 2.
constexpr double kChebHi = 2.0, kChebLo = 0.2;

// Largest coarsest level the separable direct solve takes (dense x-eigenbasis
// of nx^2 doubles, row transforms staged in LDS).
constexpr int kMgCoarseMaxNx = 2048;
constexpr int kMgCoarseMaxNy = 2048;

// One level of the hierarchy. Level 0 is the problem's grid; its right-hand
// side is the PCG residual and its output the preconditioned residual z.
struct MgLevel {
  int nx = 0, ny = 0;
  int R = 2, P = 0;           // tile rows per wavefront and workgroups per solve
  Coef c{};                   // operator coefficients (level 0: the problem's)
  void* dev_coef = nullptr;   // coefficient block owned by levels >= 1
  float* b = nullptr;         // [nb][N] right-hand side (levels >= 1)
  float* x = nullptr;         // [nb][N] approximate solution (levels >= 1)
  float* y = nullptr;         // [nb][N] x after the first post-smoothing step (levels >= 1): the
                              // post-smoothing kernels read x on a halo, so they never write in place
  float* d = nullptr;         // [nb][N] Chebyshev direction of the post-smoothing
};

struct MgData {
  uint64_t uid = 0;  // process-unique build id (cached graphs key on it, not on the address)
  int L = 0, nb = 0, R0 = 0;
  std::vector<MgLevel> lv;
  // Coarsest level: A_c = T_x (x) H_y + H_x (x) T_y is diagonalised by the
  // generalised eigenvectors of both axes, T_x phi = lam H_x phi
  // (phi^T H_x phi = 1) and T_y psi = mu H_y psi (psi^T H_y psi = 1):
  // (Phi (x) Psi)^T A_c (Phi (x) Psi) = Lam (x) I + I (x) Mu, so
  // A_c^+ b = (Phi (x) Psi) diag(1 / (lam_k + mu_j)) (Phi (x) Psi)^T b with the
  // constant mode (k = j = 0) dropped.
  int nxc = 0, nyc = 0;
  double* phi = nullptr;   // [nxc][nxc] phi[i][k]
  double* phiT = nullptr;  // [nxc][nxc] phiT[k][i]
  double* psi = nullptr;   // [nyc][nyc] psi[j'][j]
  double* psiT = nullptr;  // [nyc][nyc] psiT[j][j'] = psi[j'][j]
  double* dinv = nullptr;  // [nyc][nxc] 1 / (lam_k + mu_j), 0 for the constant mode
  double* bh = nullptr;    // [nb][nyc][nxc] transformed right-hand side, then the mode solutions
  double* bpart = nullptr; // [nb][bP] partial sums of the coarsest right-hand side
  int bP = 0;
  double* xpart = nullptr; // [nb][nyc] row sums of the coarsest solution
  float* z = nullptr;      // [nb][N0] output of the V-cycle on the fine level
  float* d0 = nullptr;     // [nb][N0] post-smoothing direction on the fine level
  float* y0 = nullptr;     // [nb][N0] fine-level x after the first post-smoothing step
  std::vector<void*> owned;
};

// Builds (or reuses) the hierarchy of L levels for nb right-hand sides, with
// the fine level tiled at R0 rows per wavefront.
ppe_status mg_ensure(ppe_problem* p, int L, int nb, int R0, hipStream_t s);
void mg_free(MgData* m);

}  // namespace ppe
