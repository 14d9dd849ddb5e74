// The plan object behind the opaque sem_plan handle.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>

#include "../../include/sem.h"
#include "plan_host.h"

struct sem_plan {
  int device = -1;
  int k = 0;
  int ne[3] = {0, 0, 0};
  int dims[3] = {0, 0, 0};
  int ld[3] = {0, 0, 0};  // padded factor dimension (multiple of 128)
  double box[6] = {0, 0, 0, 0, 0, 0};
  double alpha = 0.0;
  sem_bc bc[3] = {SEM_BC_DIRICHLET, SEM_BC_DIRICHLET, SEM_BC_DIRICHLET};  // per axis
  int per_mask = 0;  // bit a set: axis a is periodic
  size_t N = 0;
  semfd::AxisData ax[3];
  // FP64 device data
  double* d_gf[3] = {nullptr, nullptr, nullptr};  // forward factor F = S^T M, stored G[m][l] = F[l][m]
  double* d_gb[3] = {nullptr, nullptr, nullptr};  // backward factor S, stored G[m][l] = S[l][m]
  double* d_lam[3] = {nullptr, nullptr, nullptr};
  double* d_hb[3] = {nullptr, nullptr, nullptr};  // banded rows of H = M^{-1} K
  double* d_mass[3] = {nullptr, nullptr, nullptr};  // lumped 1D masses (inner products of PCG)
  // reflection-split FP64 factors [axis][0 = symmetric, 1 = antisymmetric block],
  // stored G[m][l] = A[l][m] (m contracted), zero-padded to fld x fld: forward
  // A = modes x representatives, backward A = representatives x modes of the block
  double* d_gff[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};
  double* d_gbf[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};
  int fld[3] = {0, 0, 0};
  double* d_lamf64[3] = {nullptr, nullptr, nullptr};  // eigenvalues in folded mode order (FP64 path)
  // low-precision factors (created on first use): [axis][0 = forward, 1 = backward],
  // layout [l][k], zero-padded to lp_ld x lp_ld
  void* lp_f32[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};
  void* lp_hi[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};
  void* lp_lo[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};
  int lp_ld[3] = {0, 0, 0};
  // reflection-split BF16 factors (hi plane, then lo plane lpf_plane elements
  // later) [axis][0 = forward, 1 = backward]: forward rows = symmetric modes from 0,
  // antisymmetric from lpf_frow2, columns = representatives; backward rows =
  // representatives (symmetric block from 0, antisymmetric from lpf_frow2),
  // columns = modes of the block; pitch lpf_ld
  void* lpf[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};
  int lpf_ld[3] = {0, 0, 0};
  int lpf_frow2[3] = {0, 0, 0};
  long lpf_plane[3] = {0, 0, 0};
  double* d_lamf[3] = {nullptr, nullptr, nullptr};  // eigenvalues in folded mode order
  int lp_ready = 0;
  // tuned launch shapes per precision (index sem_prec) and pass: FP32 tile rows,
  // BF16 tile order group (lp_tune)
  int tuned[4] = {0, 0, 0, 0};
  int tune_choice[4][6] = {};
  // execution
  hipStream_t stream = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_owned = false;
};

namespace semfd {
// Spectral multiplier of an FD application: 1 / (alpha + b1 L + b2 L^2) with L the
// sum of the three 1D eigenvalues (Helmholtz: {alpha, 1, 0}).
// kind / param select another multiplier of the FP64 path (EpiArgs::kind).
struct Spectral {
  double alpha, b1, b2;
  int kind = 0;
  double param = 0.0;
};
struct FoldAxis;
struct UnfoldDot;
// Buffers of the low-precision solves inside the plan workspace.
struct LpWork {
  sem_prec prec = SEM_F32;
  void* r = nullptr;        // residual / right-hand side in the intermediate format
  void* t0 = nullptr;       // rotating intermediates
  void* t1 = nullptr;
  unsigned long long* norms = nullptr;  // 2 x FP64 bit patterns
  int rkind = 1, ldr = 0;   // ResidualArgs.r_kind and row pitch of r
  long rplane = 0, tplane = 0;
  // BF16 modes: t1 already holds the folded input of the first pass (written by
  // the caller's own kernel), so the application skips its conversion
  bool input_in_t1 = false;
  // BF16 modes, first = 1: the unfold also forms these inner products
  const UnfoldDot* unfold_dot = nullptr;
};
// Geometry of the reflection split along axis a (representatives, their count
// rounded up to 32, periodic flag) and the row pitch of the z-folded BF16 input
// of the first pass.
void lp_fold_axes(const sem_plan* p, FoldAxis fa[3]);
int lp_fold_pitch_z(const sem_plan* p);
sem_status lp_prepare(sem_plan* p, sem_prec prec, LpWork* w, bool tune = true);
sem_status lp_tune(sem_plan* p, const LpWork& w);
sem_status lp_factors(sem_plan* p, sem_prec prec);
sem_status lp_layout(sem_plan* p, sem_prec prec, void* ws, LpWork* w);
hipError_t lp_fd(sem_plan* p, const LpWork& w, const Spectral& sp, const double* f64_src, double* u, int first,
                 unsigned long long* norms);
// FP64 FD application u = S_3 [g(L) (F_3 f)] on the reflection-split transforms
// (tmp: N doubles; u may alias f).
hipError_t fd64(sem_plan* p, const Spectral& sp, const double* f, double* u, double* tmp);
hipError_t zero_norms(unsigned long long* norms, hipStream_t stream);

// Refinement stop test on the relative updates r_k = ||delta_k|| / ||u_k||: met
// when r_k <= tol, or when the observed contraction, q = the larger of the last
// two ratios r_k / r_{k-1} and r_{k-1} / r_{k-2} (from the third iteration on;
// the convergence of the coarsest precisions alternates between fast and slow
// steps), is below 1/2 and makes the predicted remaining error q r_k / (1 - q)
// (the next update and all later ones for contraction q) <= tol / 10: q is an
// estimate from two ratios, not a bound, so the prediction keeps a factor of ten
// in hand.  prev = r_{k-1}, prev2 = r_{k-2}; infinite when not yet available.
inline bool refine_converged(double rel, double prev, double prev2, double tol) {
  if (!(tol > 0)) return false;
  if (rel <= tol) return true;
  if (prev > 0 && prev < 1e300 && prev2 > 0 && prev2 < 1e300) {
    const double q = fmax(rel / prev, prev / prev2);
    if (q < 0.5 && rel * q / (1.0 - q) <= 0.1 * tol) return true;
  }
  return false;
}

sem_status hip_fail(hipError_t e, const char* what);
sem_status set_error(sem_status st, const char* msg);
sem_status plan_workspace(sem_plan* p, size_t need, void** out);
size_t workspace_need(const sem_plan* p, sem_prec prec);
void release_lowp(sem_plan* p);
}  // namespace semfd
