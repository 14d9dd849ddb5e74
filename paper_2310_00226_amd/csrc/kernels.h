// Internal declarations shared by the HIP translation units of the library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace semfd {

enum { EPI_STORE = 0, EPI_DIVIDE = 1, EPI_ACCUM = 2 };

// Arguments of the fused epilogues.
//   EPI_DIVIDE: out = acc / (alpha + b1 L + b2 L^2),  L = lx[row] + ly[col / nz] + lz[col % nz]
//               (Helmholtz: b1 = 1, b2 = 0; the Cahn-Hilliard operator a + m dt eps L^2:
//               b1 = 0, b2 = m dt eps)
//   EPI_ACCUM : out += acc
struct EpiArgs {
  const double* lx = nullptr;
  const double* ly = nullptr;
  const double* lz = nullptr;
  double alpha = 0.0, b1 = 1.0, b2 = 0.0;
  long nz = 1;
};

// Denominator of the spectral divide, FP64.
__host__ __device__ inline double spectral_den(double lam, double alpha, double b1, double b2) {
  return alpha + lam * (b1 + b2 * lam);
}

// One FP64 mode product along `axis` of a row-major (dims[0], dims[1], dims[2])
// array: y[.., l, ..] = sum_m A[l][m] x[.., m, ..] with g[m * ldg + l] = A[l][m]
// (g zero-padded to a multiple of 128 in both dimensions).
hipError_t launch_mode_f64(const double* x, double* y, const double* g, int ldg, const int dims[3], int axis, int epi,
                           const EpiArgs& ea, hipStream_t stream);

// ---- low-precision rotating mode products (mode_lp.hip) ----
enum { LP_F32 = 1, LP_BF16 = 2, LP_BF16X3 = 3 };

// Epilogue arguments: divide by alpha + b1 L + b2 L^2 with L = l0[l] + l1[a] +
// l2[b] (third forward pass), or accumulate into FP64 (first = 1: u = delta)
// recording norms[0] = max|delta|, norms[1] = max|u| (bit patterns, atomic max;
// skipped when norms is null).
struct EpiLP {
  const double* l0 = nullptr;
  const double* l1 = nullptr;
  const double* l2 = nullptr;
  double alpha = 0.0, b1 = 1.0, b2 = 0.0;
  int first = 0;
  unsigned long long* norms = nullptr;
};

// One pass  Y[l][a][b] = sum_k F[l][k] X[a][b][k]:
//   x: input rows (P = A*B rows of K elements, row pitch ldx), kind in_kind
//      (0 FP64, 1 FP32, 2 BF16 bits);
//   y: output (L, A, B) with row pitch ldy, kind out_kind (1 FP32, 2 BF16, 0 FP64
//      accumulate);
//   f_hi / f_lo: factor [l][k] (FP32 or BF16 bits), padded with zeros to ldf
//      columns and to a multiple of 128 rows.
// The direct-to-LDS kernels (mode_dma.hip) take BF16 operands only: split-BF16
// operands are two planes, the second xplane / yplane / fplane elements after
// the first (f_lo unused).
struct LpPass {
  int mode = LP_BF16;
  const void* x = nullptr;
  int ldx = 0;
  long P = 0;
  int K = 0;
  void* y = nullptr;
  int ldy = 0;
  int A = 0, B = 0, L = 0;
  const void* f_hi = nullptr;
  const void* f_lo = nullptr;
  int ldf = 0;
  int in_kind = 0, out_kind = 0, epi_kind = EPI_STORE;
  long xplane = 0, yplane = 0, fplane = 0;
  EpiLP epi;
};
hipError_t launch_mode_lp(const LpPass& ps, hipStream_t stream);

// ---- BF16 / split-BF16 passes with direct global -> LDS loads (mode_dma.hip) ----
// Requirements: in_kind 2, ldx and ldf multiples of 8, ldx >= K, ldf >= L and K
// rounded up to 256; tensor pitch padding [K, ldx) holds finite values; factor
// zero outside L x K.  Output BF16 planes get their pitch padding [B, ldy) zeroed.
bool dma_supported(const LpPass& ps);
hipError_t launch_mode_dma(const LpPass& ps, hipStream_t stream);
// FP64 array (rows dims[0]*dims[1], pitch dims[2]) -> BF16 hi (+ lo plane plane_o
// elements later when split) with pitch ldo, padding zeroed.
hipError_t launch_to_lowp(const double* f, void* out, long plane_o, int split, const int dims[3], int ldo,
                          hipStream_t stream);

// Generalised nodal residual  r = cf f - cd d - ch (H_x + H_y + H_z) v  with banded
// H rows hb[a][g * (2k+1) + d] = H_a(g, g - k + d), FP64 arithmetic.
//   f == nullptr: the f term is absent;  d == nullptr: d is v itself.
//   Helmholtz residual f - alpha u - H u: (v = u, f, d = null, cf = 1, cd = alpha, ch = 1).
// r is written with row pitch ldr >= dims[2] as FP64 (r_kind 0), FP32 (1), BF16
// (2) or split BF16 (3: hi plane, lo plane rplane elements later); the pitch
// padding [dims[2], ldr) is written with zeros.  r must not alias v.
struct ResidualArgs {
  const double* v = nullptr;
  const double* f = nullptr;
  const double* d = nullptr;
  void* r = nullptr;
  int r_kind = 0;
  int ldr = 0;
  long rplane = 0;
  double cf = 1.0, cd = 0.0, ch = 1.0;
};
hipError_t launch_residual(const ResidualArgs& ra, const double* const hb[3], int k, const int dims[3],
                           hipStream_t stream);

}  // namespace semfd
