// FP64 matrix-free SEM residual.
//
// r = f - M_3^{-1} A u with A = K(x)M(x)M + M(x)K(x)M + M(x)M(x)K + alpha M(x)M(x)M
// (paper Sec. 2.4, eq. matvec3D, in the H-form of eqs. weak2D-2 / matvec2D-3
// extended to 3D):  r = f - alpha u - (H_x + H_y + H_z) u,  H = M^{-1} K per axis.
// H is banded with half-bandwidth k (a node only couples to the nodes of the
// elements it belongs to); the plan stores its rows densely as
// hb[g * (2k+1) + d] = H(g, g - k + d), zero outside the matrix.
//
// The kernels evaluate the general form  r = cf f - cd d - ch H_3 v  (see
// ResidualArgs), which also gives H_3 v alone and the residual of the
// Cahn-Hilliard operator a I + c H_3^2 in two passes.
//
// Periodic conditions (bit a of `per` for axis a): H_a couples node g through
// offset d - k to node (g - k + d) mod n_a; the kernels read v at the wrapped
// indices along that axis (the plan's band rows hold the wrap-around couplings).
//
// HBM-bound: per node it reads v and f and writes r (24 bytes in FP64).  For
// k <= 8 a block of 8 waves owns a 16 (y) x 64 (z) column of nodes and marches
// along x (residual_march_kernel): per x-plane the (16 + 2k) x (64 + 2k) tile of
// v (core and a halo of k nodes in y and z) is staged in LDS, double-buffered with
// one barrier per plane (the core from the thread's x-window registers, the halo
// from global memory, mostly L2 hits); the y and z sums read the tile, the x sum
// reads a register window of the 2k + 1 planes along x, whose front is loaded
// one plane ahead.  The z-band coefficients of a thread's column stay in
// registers (in LDS for the weighted variant), the y and x band rows are read
// per plane.  x is cut into chunks so that thin (y, z) planes still fill the
// chip.  Other k use a plain kernel with one thread per node.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "kernels.h"

namespace semfd {

namespace {

// Stores of one residual value; BF16 with a nonzero plane offset stores the split
// pair (hi at i, lo = v - hi at i + plane).
__device__ __forceinline__ void put(double* r, size_t i, double v, long) { r[i] = v; }
__device__ __forceinline__ void put(float* r, size_t i, double v, long) { r[i] = (float)v; }
__device__ __forceinline__ void put(unsigned short* r, size_t i, double v, long plane) {
  const float fv = (float)v;
  const __bf16 h = (__bf16)fv;
  r[i] = __builtin_bit_cast(unsigned short, h);
  if (plane) r[i + plane] = __builtin_bit_cast(unsigned short, (__bf16)(fv - (float)h));
}
// zero the pitch padding [nz, ldr) of one row, spread over the row's nodes: node
// l writes element l + (ldr - nz) when that lies in the padding; the last node
// also writes the part of a padding wider than the row
template <class TR>
__device__ __forceinline__ void zero_pad(TR* r, size_t row0, int l, int nz, int ldr, long plane) {
  const int npad = ldr - nz;
  if (l + npad >= nz) put(r, row0 + l + npad, 0.0, plane);
  if (l == nz - 1)
    for (int e = nz; e < npad; ++e) put(r, row0 + e, 0.0, plane);
}

// r = cf f - cd (wa + wt) (d or v) - ch H_3 v  (weight 1 without wt)
struct Coef {
  double cf, cd, ch, wa;
};

// Optional fused inner product of the weighted march: per-block partial sums of
// <v, r>_M at partial[2 b] (partial == nullptr: none).
struct DotOut {
  const double *mx = nullptr, *my = nullptr, *mz = nullptr;
  double* partial = nullptr;
};

// Generic kernel (any k): one thread per node.
template <class TR>
__global__ __launch_bounds__(256) void residual_any_kernel(const double* __restrict__ v, const double* __restrict__ f,
                                                           const double* __restrict__ dg,
                                                           const double* __restrict__ wt, TR* __restrict__ r, int ldr,
                                                           long rplane, const double* __restrict__ hx,
                                                           const double* __restrict__ hy,
                                                           const double* __restrict__ hz, int k, int nx, int ny,
                                                           int nz, int per, Coef c) {
  const int bw = 2 * k + 1;
  const long jl = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long plane = (long)ny * nz;
  if (jl >= plane) return;
  const int i = blockIdx.y;
  const int j = (int)(jl / nz);
  const int l = (int)(jl - (long)j * nz);
  const size_t idx = (size_t)i * plane + jl;
  double s = 0.0;
  {
    const double* hrow = hz + (size_t)l * bw;
    if (per & 4) {
      const size_t zrow = idx - l;  // node (i, j, 0)
      for (int d = 0; d < bw; ++d) s += hrow[d] * v[zrow + (((l - k + d) % nz) + nz) % nz];
    } else {
      const int d0 = l - k < 0 ? k - l : 0;
      const int d1 = l + k >= nz ? k + (nz - 1 - l) : 2 * k;
      for (int d = d0; d <= d1; ++d) s += hrow[d] * v[idx + (d - k)];
    }
  }
  {
    const double* hrow = hy + (size_t)j * bw;
    if (per & 2) {
      const size_t ycol = idx - (size_t)j * nz;  // node (i, 0, l)
      for (int d = 0; d < bw; ++d) s += hrow[d] * v[ycol + (size_t)((((j - k + d) % ny) + ny) % ny) * nz];
    } else {
      const int d0 = j - k < 0 ? k - j : 0;
      const int d1 = j + k >= ny ? k + (ny - 1 - j) : 2 * k;
      for (int d = d0; d <= d1; ++d) s += hrow[d] * v[idx + (long)(d - k) * nz];
    }
  }
  {
    const double* hrow = hx + (size_t)i * bw;
    if (per & 1) {
      for (int d = 0; d < bw; ++d) s += hrow[d] * v[(size_t)((((i - k + d) % nx) + nx) % nx) * plane + jl];
    } else {
      const int d0 = i - k < 0 ? k - i : 0;
      const int d1 = i + k >= nx ? k + (nx - 1 - i) : 2 * k;
      for (int d = d0; d <= d1; ++d) s += hrow[d] * v[idx + (long)(d - k) * plane];
    }
  }
  const double dv = (dg ? dg[idx] : v[idx]) * (wt ? c.wa + wt[idx] : 1.0);
  const double fv = f ? f[idx] : 0.0;
  const size_t row0 = ((size_t)i * ny + j) * ldr;
  put(r, row0 + l, c.cf * fv - c.cd * dv - c.ch * s, rplane);
  zero_pad(r, row0, l, nz, ldr, rplane);
}

// Tiled march: a block (8 waves) owns a TY (y) x TZ (z) column of nodes and marches
// along x; each wave owns RW rows of y.
constexpr int RT = 512;                       // threads per block (8 waves)
constexpr int TY = 16, TZ = 64, RW = TY / 8;  // RW rows of y per wave
constexpr int RY = TY, RZ = TZ;               // grid granularity

template <int KH>
struct TileGeo {
  static constexpr int ROWS = TY + 2 * KH, COLS = TZ + 2 * KH, PLANE = ROWS * COLS;
  // halo cells of a plane tile: KH rows above and below (full width), KH columns
  // left and right of the core rows
  static constexpr int HALO = 2 * KH * COLS + TY * 2 * KH;
  static constexpr int NH = (HALO + RT - 1) / RT;  // per thread
};

// One block's march.  Per x-plane i the tile (core + halo of KH nodes in y and z)
// of v is staged in LDS (double-buffered, one barrier per plane): the core from
// the x-window registers, the halo from global memory (neighbouring blocks' cores,
// mostly cached).  The y and z neighbour sums read the tile, the x sum reads the
// thread's register window of 2 KH + 1 planes, whose front is loaded from global
// memory one plane ahead.  Out-of-domain values are zero in the tile and the
// window (their band coefficients are zero as well).
template <int KH, class TR, bool W>
__device__ __forceinline__ void march_body(const double* __restrict__ v, const double* __restrict__ f,
                                           const double* __restrict__ dg, const double* __restrict__ wt,
                                           TR* __restrict__ r, int ldr, long rplane,
                                           const double* __restrict__ hx, const double* __restrict__ hy,
                                           const double* __restrict__ hz, int nx, int ny, int nz, int xchunk,
                                           int per, const Coef& c, int bx, int by, int bz,
                                           double* __restrict__ lds, const DotOut& dot = DotOut()) {
  constexpr int BW = 2 * KH + 1;
  typedef TileGeo<KH> G;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int z0 = bx * TZ, y0 = by * TY;
  const int l = z0 + lane;
  const bool lok = l < nz;
  const int i0 = bz * xchunk;
  const int i1 = min(nx, i0 + xchunk);
  const long plane = (long)ny * nz;
  const bool has_f = f != nullptr, has_d = dg != nullptr;  // uniform
  // ok: the thread's node exists and gets an output; ld: its tile cell holds a
  // value of v (periodic: every cell, read at the wrapped node); so: the in-plane
  // offset of that value
  int jr[RW], so[RW];
  bool ok[RW], ld[RW];
  const bool px = per & 1, py = per & 2, pz = per & 4;  // uniform
  const int ls = pz ? l % nz : l;
#pragma unroll
  for (int q = 0; q < RW; ++q) {
    jr[q] = y0 + RW * wave + q;  // wave-uniform
    ok[q] = lok && jr[q] < ny;
    ld[q] = (lok || pz) && (jr[q] < ny || py);
    so[q] = ld[q] ? (py ? jr[q] % ny : jr[q]) * nz + ls : 0;
  }
  // z-band coefficients of the thread's column: registers, or (weighted variant,
  // whose registers would otherwise hold one block per CU) an LDS row per lane
  // after the two plane tiles, written by wave 0 before the first barrier
  double cz[W ? 1 : BW];
  double* __restrict__ czl = lds + 2 * G::PLANE;
  if constexpr (W) {
    if (wave == 0)
#pragma unroll
      for (int d = 0; d < BW; ++d) czl[d * 64 + lane] = lok ? hz[(size_t)l * BW + d] : 0.0;
  } else {
#pragma unroll
    for (int d = 0; d < BW; ++d) cz[d] = lok ? hz[(size_t)l * BW + d] : 0.0;
  }
  // halo cells of this thread: LDS index and in-plane global offset (-1: outside)
  int hl[G::NH], hg[G::NH];
#pragma unroll
  for (int h = 0; h < G::NH; ++h) {
    const int idx = tid + RT * h;
    int row = 0, col = 0;
    if (idx < 2 * KH * G::COLS) {
      const int rb = idx / G::COLS;
      row = rb < KH ? rb : rb + TY;
      col = idx % G::COLS;
    } else {
      const int sdx = idx - 2 * KH * G::COLS;
      row = KH + sdx / (2 * KH);
      const int cs = sdx % (2 * KH);
      col = cs < KH ? cs : cs + TZ;
    }
    int gy = y0 - KH + row, gz = z0 - KH + col;
    if (py) gy = ((gy % ny) + ny) % ny;
    if (pz) gz = ((gz % nz) + nz) % nz;
    const bool inside = gy >= 0 && gy < ny && gz >= 0 && gz < nz;
    const bool in = idx < G::HALO;
    hl[h] = in ? row * G::COLS + col : -1;
    hg[h] = (in && inside) ? gy * nz + gz : -1;
  }
  auto at = [&](int i, int q) -> size_t { return (size_t)i * plane + (size_t)so[q]; };
  // x windows: w[q][d] = v[i - KH + d] at (jr[q], l), zero outside the domain
  double w[RW][BW];
#pragma unroll
  for (int q = 0; q < RW; ++q)
#pragma unroll
    for (int d = 0; d < BW; ++d) {
      int ii = i0 - KH + d;
      if (px) ii = ((ii % nx) + nx) % nx;
      const bool in = ld[q] && ii >= 0 && ii < nx;
      const double x = v[in ? at(ii, q) : 0];
      w[q][d] = in ? x : 0.0;
    }
  // prefetched operands of the current plane
  double hv[G::NH], fv[RW], dv[RW], wv[W ? RW : 1], wn[RW];
  auto prefetch = [&](int i) {  // halo and f/d of plane i, window front v[i + KH]
    const int ic = i < nx ? i : nx - 1;
#pragma unroll
    for (int h = 0; h < G::NH; ++h) {
      const double x = v[(size_t)ic * plane + (hg[h] >= 0 ? hg[h] : 0)];
      hv[h] = hg[h] >= 0 ? x : 0.0;
    }
    int inext = i + KH;  // enters the window when plane i - 1 is done
    if (px && inext >= nx) inext %= nx;
#pragma unroll
    for (int q = 0; q < RW; ++q) {
      const bool in = ld[q] && inext < nx;
      const double x = v[in ? at(inext, q) : 0];
      wn[q] = in ? x : 0.0;
      fv[q] = (has_f && ok[q]) ? f[at(ic, q)] : 0.0;
      dv[q] = (has_d && ok[q]) ? dg[at(ic, q)] : 0.0;
      if constexpr (W) wv[q] = ok[q] ? c.wa + wt[at(ic, q)] : 1.0;
    }
  };
  const bool fuse = W && dot.partial != nullptr;  // uniform
  double acc = 0.0;
  if (i0 < i1) prefetch(i0);
  for (int i = i0; i < i1; ++i) {
    double* __restrict__ T = lds + ((i - i0) & 1) * G::PLANE;
#pragma unroll
    for (int q = 0; q < RW; ++q) T[(KH + RW * wave + q) * G::COLS + KH + lane] = w[q][KH];
#pragma unroll
    for (int h = 0; h < G::NH; ++h)
      if (hl[h] >= 0) T[hl[h]] = hv[h];
    double fc[RW], dc[RW];
#pragma unroll
    for (int q = 0; q < RW; ++q) {
      fc[q] = fv[q];
      dc[q] = has_d ? dv[q] : w[q][KH];
      if constexpr (W) dc[q] *= wv[q];
    }
    __syncthreads();  // the plane-i tile is complete (and plane i-2's readers are done)
    prefetch(i + 1);  // halo, f, d of plane i + 1 and the window front v[i + 1 + KH]
    const double* __restrict__ hxr = hx + (size_t)i * BW;
#pragma unroll
    for (int q = 0; q < RW; ++q) {
      const int rc = KH + RW * wave + q;
      const double* __restrict__ hyr = hy + (size_t)(jr[q] < ny ? jr[q] : 0) * BW;
      double s = 0.0;
#pragma unroll
      for (int d = 0; d < BW; ++d) {
        s += hxr[d] * w[q][d];
        s += hyr[d] * T[(rc - KH + d) * G::COLS + KH + lane];
        if constexpr (W) s += czl[d * 64 + lane] * T[rc * G::COLS + lane + d];
        else s += cz[d] * T[rc * G::COLS + lane + d];
      }
      if (ok[q]) {
        const size_t row0 = ((size_t)i * ny + jr[q]) * ldr;
        const double o = c.cf * fc[q] - c.cd * dc[q] - c.ch * s;
        put(r, row0 + l, o, rplane);
        zero_pad(r, row0, l, nz, ldr, rplane);
        if constexpr (W)
          if (fuse) acc += (dot.mx[i] * dot.my[jr[q]] * dot.mz[l]) * (w[q][KH] * o);
      }
#pragma unroll
      for (int d = 0; d + 1 < BW; ++d) w[q][d] = w[q][d + 1];
      w[q][BW - 1] = wn[q];
    }
  }
  if constexpr (W) {
    if (fuse) {  // block sum in a fixed order: waves, then the 8 wave sums
      __syncthreads();  // every wave is done with the plane tiles
      for (int sh = 32; sh >= 1; sh >>= 1) acc += __shfl_xor(acc, sh);
      if (lane == 0) lds[wave] = acc;
      __syncthreads();
      if (tid == 0) {
        double t = 0.0;
        for (int k = 0; k < RT / 64; ++k) t += lds[k];
        dot.partial[2 * ((size_t)bx + (size_t)gridDim.x * ((size_t)by + (size_t)gridDim.y * bz))] = t;
      }
    }
  }
}

template <int KH, class TR, bool W>
__global__ __launch_bounds__(RT) void residual_march_kernel(const double* __restrict__ v,
                                                                  const double* __restrict__ f,
                                                                  const double* __restrict__ dg,
                                                                  const double* __restrict__ wt, TR* __restrict__ r,
                                                                  int ldr, long rplane,
                                                                  const double* __restrict__ hx,
                                                                  const double* __restrict__ hy,
                                                                  const double* __restrict__ hz, int nx, int ny,
                                                                  int nz, int xchunk, int per, Coef c,
                                                                  DotOut dot) {
  __shared__ double lds[2 * TileGeo<KH>::PLANE + (W ? (2 * KH + 1) * 64 : 0)];
  march_body<KH, TR, W>(v, f, dg, wt, r, ldr, rplane, hx, hy, hz, nx, ny, nz, xchunk, per, c, blockIdx.x,
                        blockIdx.y, blockIdx.z, lds, dot);
}

// The same march with at most 128 VGPRs (4 waves per SIMD, two blocks per CU).
// For k = 5 without the weight it fits without spilling (127 instead of 130
// VGPRs) and runs 10% faster (6.1 vs 6.8 ms at 1000^3); the weighted k = 5
// march would spill 44 bytes per lane and gain nothing, k = 4 fits either way.
template <int KH, class TR, bool W>
__global__ __launch_bounds__(RT) __attribute__((amdgpu_waves_per_eu(4, 8))) void residual_march_kernel_w4(
    const double* __restrict__ v, const double* __restrict__ f, const double* __restrict__ dg,
    const double* __restrict__ wt, TR* __restrict__ r, int ldr, long rplane, const double* __restrict__ hx,
    const double* __restrict__ hy, const double* __restrict__ hz, int nx, int ny, int nz, int xchunk, int per,
    Coef c, DotOut dot) {
  __shared__ double lds[2 * TileGeo<KH>::PLANE + (W ? (2 * KH + 1) * 64 : 0)];
  march_body<KH, TR, W>(v, f, dg, wt, r, ldr, rplane, hx, hy, hz, nx, ny, nz, xchunk, per, c, blockIdx.x,
                        blockIdx.y, blockIdx.z, lds, dot);
}

// Residuals of many solves (same k) in one launch: descriptor i owns blocks
// [block0_i, block0_i + gx * gy * gz) of the grid; inactive solves are skipped.
template <int KH, class TR>
__global__ __launch_bounds__(RT) void residual_march_batch(const ResDesc* __restrict__ descs, int nd,
                                                             const int* __restrict__ active) {
  __shared__ double lds[2 * TileGeo<KH>::PLANE];
  const long i = blockIdx.x;
  int lo = 0, hi = nd;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (descs[mid].block0 <= i) lo = mid;
    else hi = mid;
  }
  const ResDesc& d = descs[lo];
  if (!active[d.sid]) return;
  const long rb = i - d.block0;
  const int bx = (int)(rb % d.gx);
  const int by = (int)((rb / d.gx) % d.gy);
  const int bz = (int)(rb / ((long)d.gx * d.gy));
  march_body<KH, TR, false>(d.v, d.f, d.d, nullptr, (TR*)d.r, d.ldr, d.rplane, d.hx, d.hy, d.hz, d.nx, d.ny, d.nz,
                            d.xchunk, d.per, Coef{d.cf, d.cd, d.ch, 0.0}, bx, by, bz, lds);
}

// x is split into chunks so that the grid fills the chip even for thin (y, z)
// planes; a chunk spans at least 8 k planes, since each chunk first loads the 2k
// planes of its window
void march_grid(const int dims[3], int k, int* gx, int* gy, int* gz, int* xchunk) {
  const long cols = (long)((dims[2] + RZ - 1) / RZ) * ((dims[1] + RY - 1) / RY);
  int nchunks = (int)std::min<long>(dims[0], std::max<long>(1, (8192 + cols - 1) / cols));
  *xchunk = std::max((dims[0] + nchunks - 1) / nchunks, std::min(dims[0], 8 * k));
  *gx = (dims[2] + RZ - 1) / RZ;
  *gy = (dims[1] + RY - 1) / RY;
  *gz = (dims[0] + *xchunk - 1) / *xchunk;
}

template <int KH, class TR>
void launch_march(const ResidualArgs& ra, TR* r, const double* const hb[3], const int dims[3], Coef c,
                  hipStream_t stream) {
  int gx, gy, gz, xchunk;
  march_grid(dims, KH, &gx, &gy, &gz, &xchunk);
  // the per-node weight (an FP64 operator application of the variable-coefficient
  // solver) has its own instantiation, so that the others keep their registers
  if constexpr (std::is_same<TR, double>::value) {
    if (ra.wt) {
      DotOut dot;
      if (ra.dot_partial) dot = DotOut{ra.dot_mass[0], ra.dot_mass[1], ra.dot_mass[2], ra.dot_partial};
      if constexpr (KH == 4 || KH == 5)
        residual_march_kernel_w4<KH, TR, true><<<dim3(gx, gy, gz), dim3(RT), 0, stream>>>(
            ra.v, ra.f, ra.d, ra.wt, r, ra.ldr, ra.rplane, hb[0], hb[1], hb[2], dims[0], dims[1], dims[2], xchunk,
            ra.periodic, c, dot);
      else
        residual_march_kernel<KH, TR, true><<<dim3(gx, gy, gz), dim3(RT), 0, stream>>>(
            ra.v, ra.f, ra.d, ra.wt, r, ra.ldr, ra.rplane, hb[0], hb[1], hb[2], dims[0], dims[1], dims[2], xchunk,
            ra.periodic, c, dot);
      return;
    }
  }
  if constexpr (KH == 5) {
    residual_march_kernel_w4<KH, TR, false><<<dim3(gx, gy, gz), dim3(RT), 0, stream>>>(
        ra.v, ra.f, ra.d, nullptr, r, ra.ldr, ra.rplane, hb[0], hb[1], hb[2], dims[0], dims[1], dims[2], xchunk,
        ra.periodic, c, DotOut());
  } else {
    residual_march_kernel<KH, TR, false><<<dim3(gx, gy, gz), dim3(RT), 0, stream>>>(
        ra.v, ra.f, ra.d, nullptr, r, ra.ldr, ra.rplane, hb[0], hb[1], hb[2], dims[0], dims[1], dims[2], xchunk,
        ra.periodic, c, DotOut());
  }
}

template <int KH>
hipError_t batch_typed(int r_kind, const ResDesc* descs, int nd, long total_blocks, const int* active,
                       hipStream_t s) {
  const dim3 grid((unsigned)total_blocks), block(RT);
  switch (r_kind) {
    case 0: residual_march_batch<KH, double><<<grid, block, 0, s>>>(descs, nd, active); break;
    case 1: residual_march_batch<KH, float><<<grid, block, 0, s>>>(descs, nd, active); break;
    case 2:
    case 3: residual_march_batch<KH, unsigned short><<<grid, block, 0, s>>>(descs, nd, active); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class TR>
hipError_t launch_typed(const ResidualArgs& ra, TR* r, const double* const hb[3], int k, const int dims[3],
                        hipStream_t stream) {
  const Coef c{ra.cf, ra.cd, ra.ch, ra.wa};
  switch (k) {
    case 1: launch_march<1, TR>(ra, r, hb, dims, c, stream); break;
    case 2: launch_march<2, TR>(ra, r, hb, dims, c, stream); break;
    case 3: launch_march<3, TR>(ra, r, hb, dims, c, stream); break;
    case 4: launch_march<4, TR>(ra, r, hb, dims, c, stream); break;
    case 5: launch_march<5, TR>(ra, r, hb, dims, c, stream); break;
    case 6: launch_march<6, TR>(ra, r, hb, dims, c, stream); break;
    case 7: launch_march<7, TR>(ra, r, hb, dims, c, stream); break;
    case 8: launch_march<8, TR>(ra, r, hb, dims, c, stream); break;
    default: {
      const long plane = (long)dims[1] * dims[2];
      dim3 block(256), grid((unsigned)((plane + 255) / 256), (unsigned)dims[0]);
      residual_any_kernel<TR><<<grid, block, 0, stream>>>(ra.v, ra.f, ra.d, ra.wt, r, ra.ldr, ra.rplane, hb[0], hb[1],
                                                          hb[2], k, dims[0], dims[1], dims[2], ra.periodic, c);
    }
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_residual(const ResidualArgs& ra, const double* const hb[3], int k, const int dims[3],
                           hipStream_t stream) {
  const long plane = (long)dims[1] * dims[2];
  if (dims[0] <= 0 || plane <= 0) return hipSuccess;
  if (!ra.v || !ra.r || ra.ldr < dims[2] || k < 1) return hipErrorInvalidValue;
  if (ra.wt && ra.r_kind != 0) return hipErrorInvalidValue;  // weights: FP64 output only
  if (ra.dot_partial && (!ra.wt || k > 8)) return hipErrorInvalidValue;  // fused dot: weighted march only
  // in-plane offsets are 32-bit; the grid's y and z extents are limited to 65535
  if ((dims[1] + RY - 1) / RY > 65535 || dims[0] > 65535 || plane > 0x7fffffffL) return hipErrorInvalidValue;
  switch (ra.r_kind) {
    case 0: return launch_typed<double>(ra, (double*)ra.r, hb, k, dims, stream);
    case 1: return launch_typed<float>(ra, (float*)ra.r, hb, k, dims, stream);
    case 2: {
      ResidualArgs rb = ra;
      rb.rplane = 0;
      return launch_typed<unsigned short>(rb, (unsigned short*)ra.r, hb, k, dims, stream);
    }
    case 3:
      if (ra.rplane <= 0) return hipErrorInvalidValue;
      return launch_typed<unsigned short>(ra, (unsigned short*)ra.r, hb, k, dims, stream);
    default:
      return hipErrorInvalidValue;
  }
}

long residual_march_blocks(const int dims[3], int k) {
  if (k < 1 || k > 8 || dims[0] <= 0 || dims[1] <= 0 || dims[2] <= 0) return 0;
  int gx, gy, gz, xchunk;
  march_grid(dims, k, &gx, &gy, &gz, &xchunk);
  return (long)gx * gy * gz;
}

bool residual_desc(const ResidualArgs& ra, const double* const hb[3], int k, const int dims[3], ResDesc* d) {
  if (k < 1 || k > 8 || !ra.v || !ra.r || ra.ldr < dims[2] || dims[0] <= 0 || dims[1] <= 0 || dims[2] <= 0)
    return false;
  if (ra.wt) return false;  // the batched residual has no per-node weight
  if ((long)dims[1] * dims[2] > 0x7fffffffL) return false;
  if (ra.r_kind == 3 && ra.rplane <= 0) return false;
  d->v = ra.v;
  d->f = ra.f;
  d->d = ra.d;
  d->r = ra.r;
  d->hx = hb[0];
  d->hy = hb[1];
  d->hz = hb[2];
  d->rplane = ra.r_kind == 3 ? ra.rplane : 0;
  d->ldr = ra.ldr;
  d->nx = dims[0];
  d->ny = dims[1];
  d->nz = dims[2];
  march_grid(dims, k, &d->gx, &d->gy, &d->gz, &d->xchunk);
  d->cf = ra.cf;
  d->cd = ra.cd;
  d->ch = ra.ch;
  d->per = ra.periodic;
  return true;
}

hipError_t launch_residual_batch(int k, int r_kind, const ResDesc* descs, int nd, long total_blocks,
                                 const int* active, hipStream_t stream) {
  if (nd <= 0 || total_blocks <= 0) return hipSuccess;
  if (total_blocks > 0x7fffffffL) return hipErrorInvalidValue;
  switch (k) {
    case 1: return batch_typed<1>(r_kind, descs, nd, total_blocks, active, stream);
    case 2: return batch_typed<2>(r_kind, descs, nd, total_blocks, active, stream);
    case 3: return batch_typed<3>(r_kind, descs, nd, total_blocks, active, stream);
    case 4: return batch_typed<4>(r_kind, descs, nd, total_blocks, active, stream);
    case 5: return batch_typed<5>(r_kind, descs, nd, total_blocks, active, stream);
    case 6: return batch_typed<6>(r_kind, descs, nd, total_blocks, active, stream);
    case 7: return batch_typed<7>(r_kind, descs, nd, total_blocks, active, stream);
    case 8: return batch_typed<8>(r_kind, descs, nd, total_blocks, active, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace semfd
