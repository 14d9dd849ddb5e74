// Reflection fold and unfold of FP64 arrays along one axis, for the FP64 solve on
// the reflection-split transforms.
//
// On a uniform mesh the reflection of an axis maps node i to R(i) = n - 1 - i
// (Dirichlet, Neumann) or (n - i) mod n (periodic) and commutes with the 1D
// stiffness and mass, so the 1D eigenvectors are symmetric or antisymmetric and
// every transform splits into two half-size blocks acting on
//     v+_r = v_r + v_R(r),   v-_r = v_r - v_R(r),   r < nrep
// (nrep = ceil(n / 2), periodic n / 2 + 1: one representative per orbit).  Viewing
// a row-major array as X[p][i][q] (p: outer axes, i: the axis, q: inner axes of
// extent Q), the folded array is Y[p][s][q] with s < 2 nrep:
//     fold:    Y[p][r] = X[p][r] + X[p][R(r)],   Y[p][nrep + r] = X[p][r] - X[p][R(r)]
//     unfold:  X[p][r] = Y[p][r] + Y[p][nrep + r],   X[p][R(r)] = Y[p][r] - Y[p][nrep + r]
// (the second unfold assignment only where R(r) != r; for such fixed nodes the
// antisymmetric part is zero).  HBM-bound: 8 bytes in and out per element.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace semfd {

namespace {

constexpr int FT = 256;  // threads per block
constexpr int FU = 4;    // elements per thread and round (loads in flight before the stores)

__device__ __forceinline__ int refl(int r, int n, int per) { return per ? (n - r) % n : n - 1 - r; }

// Blocks stride over rows: (p, r) when Q > 1 (threads over q), p when Q == 1
// (threads over r).
__global__ __launch_bounds__(FT) void fold_f64_kernel(const double* __restrict__ x, double* __restrict__ y, long P,
                                                      int n, long Q, int nrep, int per, int unfold) {
  const long nr2 = 2L * nrep;
  if (Q > 1) {
    const long rows = P * nrep;
    for (long row = blockIdx.x; row < rows; row += gridDim.x) {
      const long p = row / nrep;
      const int r = (int)(row - p * nrep), m = refl(r, n, per);
      const double* __restrict__ xa = unfold ? x + (size_t)(p * nr2 + r) * Q : x + (size_t)(p * n + r) * Q;
      const double* __restrict__ xb = unfold ? x + (size_t)(p * nr2 + nrep + r) * Q : x + (size_t)(p * n + m) * Q;
      double* __restrict__ ya = unfold ? y + (size_t)(p * n + r) * Q : y + (size_t)(p * nr2 + r) * Q;
      double* __restrict__ yb = unfold ? y + (size_t)(p * n + m) * Q : y + (size_t)(p * nr2 + nrep + r) * Q;
      const bool second = !unfold || m != r;  // uniform over the block
      for (long q0 = threadIdx.x; q0 < Q; q0 += FT * FU) {
        double a[FU], b[FU];
#pragma unroll
        for (int u = 0; u < FU; ++u) {
          const long q = q0 + (long)FT * u;
          a[u] = q < Q ? xa[q] : 0.0;
          b[u] = q < Q ? xb[q] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < FU; ++u) {
          const long q = q0 + (long)FT * u;
          if (q < Q) {
            ya[q] = a[u] + b[u];
            if (second) yb[q] = a[u] - b[u];
          }
        }
      }
    }
  } else {
    for (long p = blockIdx.x; p < P; p += gridDim.x) {
      const double* __restrict__ xp = x + (size_t)p * (unfold ? nr2 : n);
      double* __restrict__ yp = y + (size_t)p * (unfold ? n : nr2);
      for (int r0 = threadIdx.x; r0 < nrep; r0 += FT * FU) {
        double a[FU], b[FU];
#pragma unroll
        for (int u = 0; u < FU; ++u) {
          const int r = r0 + FT * u;
          const int rr = r < nrep ? r : nrep - 1;
          a[u] = xp[rr];
          b[u] = unfold ? xp[nrep + rr] : xp[refl(rr, n, per)];
        }
#pragma unroll
        for (int u = 0; u < FU; ++u) {
          const int r = r0 + FT * u;
          if (r >= nrep) continue;
          if (unfold) {
            const int m = refl(r, n, per);
            yp[r] = a[u] + b[u];
            if (m != r) yp[m] = a[u] - b[u];
          } else {
            yp[r] = a[u] + b[u];
            yp[nrep + r] = a[u] - b[u];
          }
        }
      }
    }
  }
}

}  // namespace

hipError_t launch_fold_f64(const double* x, double* y, long P, int n, long Q, int nrep, int per, int unfold,
                           hipStream_t stream) {
  if (P <= 0 || Q <= 0 || n <= 0) return hipSuccess;
  if (nrep < 1 || nrep > n || 2 * nrep < n) return hipErrorInvalidValue;
  const long rows = Q > 1 ? P * nrep : P;
  const long grid = rows < 16384 ? rows : 16384;
  fold_f64_kernel<<<dim3((unsigned)grid), dim3(FT), 0, stream>>>(x, y, P, n, Q, nrep, per, unfold);
  return hipGetLastError();
}

}  // namespace semfd
