// FP64 matrix-free SEM residual.
//
// r = f - M_3^{-1} A u with A = K(x)M(x)M + M(x)K(x)M + M(x)M(x)K + alpha M(x)M(x)M
// (paper Sec. 2.4, eq. matvec3D, in the H-form of eqs. weak2D-2 / matvec2D-3
// extended to 3D):  r = f - alpha u - (H_x + H_y + H_z) u,  H = M^{-1} K per axis.
// H is banded with half-bandwidth k (a node only couples to the nodes of the
// elements it belongs to); the plan stores its rows densely as
// hb[g * (2k+1) + d] = H(g, g - k + d), zero outside the matrix.
//
// HBM-bound: per node it reads u and f and writes r (24 bytes).  A block owns a
// (4 y) x (64 z) column of nodes and marches along x: the 2k+1 values of u along
// x that a node needs sit in a register window (each u value is loaded once, as
// the window front), the y and z neighbours of the current plane come through
// the L1 cache, and the band coefficients of H_y, H_z of the thread's (j, l)
// stay in registers for the whole march.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace semfd {

__device__ __forceinline__ void put(double* r, size_t i, double v) { r[i] = v; }
__device__ __forceinline__ void put(float* r, size_t i, double v) { r[i] = (float)v; }
__device__ __forceinline__ void put(unsigned short* r, size_t i, double v) {
  r[i] = __builtin_bit_cast(unsigned short, (__bf16)(float)v);
}

// r is written with row pitch ldr (>= nz) in type TR: FP64 for sem_residual,
// FP32 / BF16 when it only feeds a low-precision solve (refinement).
template <int KH, class TR>
__global__ __launch_bounds__(256) void residual_f64_kernel(const double* __restrict__ u, const double* __restrict__ f,
                                                           TR* __restrict__ r, int ldr, const double* __restrict__ hx,
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
  put(r, ((size_t)i * ny + j) * ldr + l, f[idx] - s);
}

constexpr int RY = 4, RZ = 64;

template <int KH, class TR>
__global__ __launch_bounds__(RY * RZ) void residual_march_kernel(const double* __restrict__ u,
                                                                  const double* __restrict__ f, TR* __restrict__ r,
                                                                  int ldr, const double* __restrict__ hx,
                                                                  const double* __restrict__ hy,
                                                                  const double* __restrict__ hz, int nx, int ny,
                                                                  int nz, int xchunk, double alpha) {
  constexpr int BW = 2 * KH + 1;
  const int l = blockIdx.x * RZ + (threadIdx.x % RZ);
  const int j = blockIdx.y * RY + (threadIdx.x / RZ);
  const int i0 = blockIdx.z * xchunk;
  const int i1 = min(nx, i0 + xchunk);
  if (l >= nz || j >= ny) return;  // no barriers below: early exit is safe
  const long plane = (long)ny * nz;
  const long col = (long)j * nz + l;
  double cy[BW], cz[BW];
#pragma unroll
  for (int d = 0; d < BW; ++d) {
    cy[d] = hy[(size_t)j * BW + d];
    cz[d] = hz[(size_t)l * BW + d];
  }
  // neighbour validity along y and z (fixed for the march)
  bool oky[BW], okz[BW];
#pragma unroll
  for (int d = 0; d < BW; ++d) {
    oky[d] = j - KH + d >= 0 && j - KH + d < ny;
    okz[d] = l - KH + d >= 0 && l - KH + d < nz;
  }
  // x window: w[d] = u[i - KH + d], zero outside [0, nx)
  double w[BW];
#pragma unroll
  for (int d = 0; d < BW; ++d) {
    const int ii = i0 - KH + d;
    w[d] = (ii >= 0 && ii < nx) ? u[(size_t)ii * plane + col] : 0.0;
  }
  for (int i = i0; i < i1; ++i) {
    const size_t idx = (size_t)i * plane + col;
    const double* __restrict__ hxr = hx + (size_t)i * BW;
    double s = alpha * w[KH];
#pragma unroll
    for (int d = 0; d < BW; ++d) s += hxr[d] * w[d];
#pragma unroll
    for (int d = 0; d < BW; ++d)
      if (oky[d]) s += cy[d] * u[idx + (long)(d - KH) * nz];
#pragma unroll
    for (int d = 0; d < BW; ++d)
      if (okz[d]) s += cz[d] * u[idx + (d - KH)];
    put(r, ((size_t)i * ny + j) * ldr + l, f[idx] - s);
    // advance the window
#pragma unroll
    for (int d = 0; d + 1 < BW; ++d) w[d] = w[d + 1];
    const int inext = i + KH + 1;
    w[BW - 1] = inext < nx ? u[(size_t)inext * plane + col] : 0.0;
  }
}

template <int KH, class TR>
static void launch_march(const double* u, const double* f, TR* r, int ldr, const double* const hb[3],
                         const int dims[3], double alpha, hipStream_t stream) {
  // split x into chunks so that the grid fills the chip even for thin (y, z) planes
  const long cols = (long)((dims[2] + RZ - 1) / RZ) * ((dims[1] + RY - 1) / RY);
  int nchunks = (int)std::min<long>(dims[0], std::max<long>(1, (2048 + cols - 1) / cols));
  const int xchunk = (dims[0] + nchunks - 1) / nchunks;
  nchunks = (dims[0] + xchunk - 1) / xchunk;
  dim3 grid((unsigned)((dims[2] + RZ - 1) / RZ), (unsigned)((dims[1] + RY - 1) / RY), (unsigned)nchunks);
  residual_march_kernel<KH, TR><<<grid, dim3(RY * RZ), 0, stream>>>(u, f, r, ldr, hb[0], hb[1], hb[2], dims[0],
                                                                     dims[1], dims[2], xchunk, alpha);
}

template <class TR>
static hipError_t launch_res(const double* u, const double* f, TR* r, int ldr, const double* const hb[3], int k,
                             const int dims[3], double alpha, hipStream_t stream) {
  const long plane = (long)dims[1] * dims[2];
  if (dims[0] <= 0 || plane <= 0) return hipSuccess;
  if ((dims[1] + RY - 1) / RY > 65535 || dims[0] > 65535) return hipErrorInvalidValue;
  switch (k) {
    case 1: launch_march<1, TR>(u, f, r, ldr, hb, dims, alpha, stream); break;
    case 2: launch_march<2, TR>(u, f, r, ldr, hb, dims, alpha, stream); break;
    case 3: launch_march<3, TR>(u, f, r, ldr, hb, dims, alpha, stream); break;
    case 4: launch_march<4, TR>(u, f, r, ldr, hb, dims, alpha, stream); break;
    case 5: launch_march<5, TR>(u, f, r, ldr, hb, dims, alpha, stream); break;
    case 6: launch_march<6, TR>(u, f, r, ldr, hb, dims, alpha, stream); break;
    case 7: launch_march<7, TR>(u, f, r, ldr, hb, dims, alpha, stream); break;
    case 8: launch_march<8, TR>(u, f, r, ldr, hb, dims, alpha, stream); break;
    default: {
      dim3 block(256), grid((unsigned)((plane + 255) / 256), (unsigned)dims[0]);
      residual_f64_kernel<0, TR><<<grid, block, 0, stream>>>(u, f, r, ldr, hb[0], hb[1], hb[2], k, dims[0], dims[1],
                                                            dims[2], alpha);
    }
  }
  return hipGetLastError();
}

hipError_t launch_residual_f64(const double* u, const double* f, double* r, const double* const hb[3], int k,
                               const int dims[3], double alpha, hipStream_t stream) {
  return launch_res<double>(u, f, r, dims[2], hb, k, dims, alpha, stream);
}

hipError_t launch_residual_lp(const double* u, const double* f, void* r, int r_kind, int ldr, const double* const hb[3],
                              int k, const int dims[3], double alpha, hipStream_t stream) {
  if (r_kind == 1) return launch_res<float>(u, f, (float*)r, ldr, hb, k, dims, alpha, stream);
  if (r_kind == 2) return launch_res<unsigned short>(u, f, (unsigned short*)r, ldr, hb, k, dims, alpha, stream);
  return launch_res<double>(u, f, (double*)r, ldr, hb, k, dims, alpha, stream);
}

}  // namespace semfd
