// Internal declarations shared by the HIP translation units of the library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace semfd {

enum { EPI_STORE = 0, EPI_DIVIDE = 1, EPI_ACCUM = 2 };

// Arguments of the fused epilogues.
//   EPI_DIVIDE: out = acc / (lx[row] + ly[col / nz] + lz[col % nz] + alpha)
//   EPI_ACCUM : out += acc
struct EpiArgs {
  const double* lx = nullptr;
  const double* ly = nullptr;
  const double* lz = nullptr;
  double alpha = 0.0;
  long nz = 1;
};

// One FP64 mode product along `axis` of a row-major (dims[0], dims[1], dims[2])
// array: y[.., l, ..] = sum_m A[l][m] x[.., m, ..] with g[m * ldg + l] = A[l][m]
// (g zero-padded to a multiple of 128 in both dimensions).
hipError_t launch_mode_f64(const double* x, double* y, const double* g, int ldg, const int dims[3], int axis, int epi,
                           const EpiArgs& ea, hipStream_t stream);

// Nodal residual r = f - alpha u - (H_x + H_y + H_z) u with banded H rows
// hb[a][g * (2k+1) + d] = H_a(g, g - k + d).
hipError_t launch_residual_f64(const double* u, const double* f, double* r, const double* const hb[3], int k,
                               const int dims[3], double alpha, hipStream_t stream);

}  // namespace semfd
