// FP64 matrix-free SEM residual.
//
// r = f - M_3^{-1} A u with A = K(x)M(x)M + M(x)K(x)M + M(x)M(x)K + alpha M(x)M(x)M
// (paper Sec. 2.4, eq. matvec3D, in the H-form of eqs. weak2D-2 / matvec2D-3
// extended to 3D):  r = f - alpha u - (H_x + H_y + H_z) u,  H = M^{-1} K per axis.
// H is banded with half-bandwidth k (a node only couples to the nodes of the
// elements it belongs to); the plan stores its rows densely as
// hb[g * (2k+1) + d] = H(g, g - k + d), zero outside the matrix.
//
// HBM-bound: per node it reads u and f and writes r (24 bytes).  Neighbours
// along z come from the same cache lines, along y from rows n_z apart and along
// x from planes n_y n_z apart; both stay in L2 / MALL while a block sweeps its
// (y, z) slab.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace semfd {

template <int KH>
__global__ __launch_bounds__(256) void residual_f64_kernel(const double* __restrict__ u, const double* __restrict__ f,
                                                           double* __restrict__ r, const double* __restrict__ hx,
                                                           const double* __restrict__ hy,
                                                           const double* __restrict__ hz, int kh, int nx, int ny,
                                                           int nz, double alpha) {
  const int k = KH > 0 ? KH : kh;
  const int bw = 2 * k + 1;
  const long jl = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long plane = (long)ny * nz;
  if (jl >= plane) return;
  const int i = blockIdx.y;
  const int j = (int)(jl / nz);
  const int l = (int)(jl - (long)j * nz);
  const size_t idx = (size_t)i * plane + jl;
  double s = alpha * u[idx];
  // z (contiguous)
  {
    const double* hrow = hz + (size_t)l * bw;
    const int d0 = l - k < 0 ? k - l : 0;
    const int d1 = l + k >= nz ? k + (nz - 1 - l) : 2 * k;
    for (int d = d0; d <= d1; ++d) s += hrow[d] * u[idx + (d - k)];
  }
  // y
  {
    const double* hrow = hy + (size_t)j * bw;
    const int d0 = j - k < 0 ? k - j : 0;
    const int d1 = j + k >= ny ? k + (ny - 1 - j) : 2 * k;
    for (int d = d0; d <= d1; ++d) s += hrow[d] * u[idx + (long)(d - k) * nz];
  }
  // x
  {
    const double* hrow = hx + (size_t)i * bw;
    const int d0 = i - k < 0 ? k - i : 0;
    const int d1 = i + k >= nx ? k + (nx - 1 - i) : 2 * k;
    for (int d = d0; d <= d1; ++d) s += hrow[d] * u[idx + (long)(d - k) * plane];
  }
  r[idx] = f[idx] - s;
}

hipError_t launch_residual_f64(const double* u, const double* f, double* r, const double* const hb[3], int k,
                               const int dims[3], double alpha, hipStream_t stream) {
  const long plane = (long)dims[1] * dims[2];
  if (dims[0] <= 0 || plane <= 0) return hipSuccess;
  if (dims[0] > 65535) return hipErrorInvalidValue;
  dim3 block(256), grid((unsigned)((plane + 255) / 256), (unsigned)dims[0]);
  if (k == 4)
    residual_f64_kernel<4><<<grid, block, 0, stream>>>(u, f, r, hb[0], hb[1], hb[2], k, dims[0], dims[1], dims[2],
                                                      alpha);
  else
    residual_f64_kernel<0><<<grid, block, 0, stream>>>(u, f, r, hb[0], hb[1], hb[2], k, dims[0], dims[1], dims[2],
                                                      alpha);
  return hipGetLastError();
}

}  // namespace semfd
