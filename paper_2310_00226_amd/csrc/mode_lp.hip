// FP32 rotating mode products for the mixed-precision refinement path: one pass
// of one solve, and the same passes of many solves in one persistent launch.
//
// Each pass contracts the CONTIGUOUS axis of its input and writes the output
// with the axes rotated:  X (A, B, K) -> Y (K', A, B),
//        Y[l][a][b] = sum_k F[l][k] X[a][b][k].
// Three passes rotate (x, y, z) -> (z, x, y) -> (y, z, x) -> (x, y, z), so the
// three forward products (and the three backward ones) of eq. 3D-Poisson return
// to the caller's layout while every pass reads both MFMA operands -- factor
// rows F[l][:] and tensor rows X[p][:] -- contiguously along the contraction.
//
// GEMM view:  C[l][p] = sum_k F[l][k] X[p][k],  p = a*B + b, output address
// (l*A + a)*ldy + b.  Block tile BM (l) x BN (p) of v_mfma_f32_16x16x4_f32
// tiles, register-staged loads into a double-buffered LDS tile.  The tile
// shapes (128 x 128, 96 x 128, 64 x 128, 32 x 128) cover large and small
// contraction lengths; the batched launcher picks one per length bucket by
// timing them, the single launcher the one with the fewest padded rows.
// Epilogues: store (FP32 intermediates), spectral divide (third forward pass),
// or accumulate into the FP64 solution (u += delta) while recording max|delta|
// and max|u| for the refinement stop test.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdint>

#include "kernels.h"

namespace semfd {

typedef float f4_t __attribute__((ext_vector_type(4)));

namespace f32k {

// Block tile BM (l) x BN (p) on WL x WP waves; each wave owns a (BM/WL) x (BN/WP)
// sub-tile of 16 x 16 MFMA tiles.
template <int BM_, int BN_, int WL_, int WP_>
struct Tile {
  static constexpr int BM = BM_, BN = BN_, WL = WL_, WP = WP_;
  static constexpr int NTHREADS = 64 * WL * WP;
  static constexpr int TL = BM / WL, TP = BN / WP;  // wave tile
  static constexpr int FL = TL / 16, FP = TP / 16;  // MFMA tiles per wave
};
typedef Tile<128, 128, 2, 2> T128;  // 4 waves of 64 x 64
typedef Tile<96, 128, 2, 2> T96;    // 4 waves of 48 x 64
typedef Tile<64, 128, 2, 2> T64;    // 4 waves of 32 x 64
typedef Tile<32, 128, 1, 4> T32;    // 4 waves of 32 x 32

constexpr int BK = 32;           // contraction chunk (8 MFMA steps of 4)
constexpr int LDS_ROW = BK + 4;  // floats per LDS row (16 bytes of padding)

template <class TIn, class TT>
struct Cfg {
  static constexpr int NTHREADS = TT::NTHREADS;
  static constexpr int TILE_F = TT::BM * LDS_ROW;  // factor tile (floats)
  static constexpr int TILE_X = TT::BN * LDS_ROW;  // tensor tile (floats)
  static constexpr int STAGE = TILE_F + TILE_X;
  // tensor staging: groups of 4 consecutive contraction elements (16 bytes of
  // FP32) read as one 16-byte load, or four 8-byte loads for FP64 input (whose
  // rows may be odd-sized)
  static constexpr int G = 4;
  static constexpr int VEC_IN = sizeof(TIn) == 8 ? 1 : 4;
  static constexpr int LOADS_PER_G = G / VEC_IN;
  static constexpr int NGROUP = TT::BN * BK / G / NTHREADS;
  static constexpr int NLOAD_F = TT::BM * BK / 4 / NTHREADS;
  static_assert(NGROUP * G * NTHREADS == TT::BN * BK, "tensor tile load mapping");
  static_assert(NLOAD_F * 4 * NTHREADS == TT::BM * BK, "factor tile load mapping");
};

__device__ __forceinline__ long xcd_tile(long nblocks_padded) {
  const long per = nblocks_padded / 8;
  return (long)(blockIdx.x % 8) * per + (long)(blockIdx.x / 8);
}

// One output tile t (l-tile fastest) of the pass described by d.
template <class TIn, class TOut, int EPI, class TT>
__device__ __forceinline__ void tile_body(const LpDesc& d, long t, float* __restrict__ lds) {
  typedef Cfg<TIn, TT> C;
  constexpr int BM = TT::BM, BN = TT::BN, NTHREADS = TT::NTHREADS, FL = TT::FL, FP = TT::FP;
  constexpr int LR = LDS_ROW;
  const TIn* __restrict__ x = (const TIn*)d.x;
  TOut* __restrict__ y = (TOut*)d.y;
  const float* __restrict__ f = (const float*)d.f;
  const int ldx = d.ldx, K = d.K, ldy = d.ldy, A = d.A, B = d.B, L = d.L, ldf = d.ldf;
  const long P = d.P;
  const long lt = t % d.tiles_l;
  const long pt = t / d.tiles_l;
  const int l0 = (int)(lt * BM);
  const long p0 = pt * BN;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / TT::WP) * TT::TL;  // rows: l
  const int wn = (wave % TT::WP) * TT::TP;  // cols: p

  // ---- global load mapping: consecutive lanes take consecutive groups of a row
  constexpr int G_PER_ROW = BK / C::G;
  constexpr int FV_PER_ROW = BK / 4;
  const TIn* __restrict__ xb = x + (size_t)p0 * ldx;
  const int prow_max = (int)(P - 1 - p0);

  typedef TIn xvec_t __attribute__((ext_vector_type(C::VEC_IN)));
  xvec_t rx[C::NGROUP][C::LOADS_PER_G];
  f4_t rf[C::NLOAD_F];
  const int nchunk = (K + BK - 1) / BK;

  auto load_chunk = [&](int c) {
    const int k0 = c * BK;
#pragma unroll
    for (int g = 0; g < C::NGROUP; ++g) {
      const int idx = g * NTHREADS + tid;
      const int row = idx / G_PER_ROW;
      const int kg = (idx % G_PER_ROW) * C::G;
      const int rr = row < prow_max ? row : prow_max;
      const TIn* __restrict__ src = xb + (size_t)rr * ldx;
#pragma unroll
      for (int v = 0; v < C::LOADS_PER_G; ++v) {
        const int kk = k0 + kg + v * C::VEC_IN;
        // past the row end: any valid address (zeroed at store time)
        rx[g][v] = *reinterpret_cast<const xvec_t*>(src + (kk < K ? kk : 0));
      }
    }
#pragma unroll
    for (int v = 0; v < C::NLOAD_F; ++v) {
      const int idx = v * NTHREADS + tid;
      const int row = idx / FV_PER_ROW;
      const int kk = (idx % FV_PER_ROW) * 4;
      // factor zero-padded to ldf x ldf (multiple of 256): always in bounds
      rf[v] = *reinterpret_cast<const f4_t*>(f + (size_t)(l0 + row) * ldf + k0 + kk);
    }
  };

  auto store_chunk = [&](int buf, int c) {
    float* sf = lds + buf * C::STAGE;
    float* sx = sf + C::TILE_F;
    const int k0 = c * BK;
    const bool tail = k0 + BK > K;  // uniform: only the last chunk
#pragma unroll
    for (int v = 0; v < C::NLOAD_F; ++v) {
      const int idx = v * NTHREADS + tid;
      const int row = idx / FV_PER_ROW;
      const int kk = (idx % FV_PER_ROW) * 4;
      *reinterpret_cast<f4_t*>(sf + row * LR + kk) = rf[v];
    }
#pragma unroll
    for (int g = 0; g < C::NGROUP; ++g) {
      const int idx = g * NTHREADS + tid;
      const int row = idx / G_PER_ROW;
      const int kg = (idx % G_PER_ROW) * C::G;
      f4_t w;
#pragma unroll
      for (int v = 0; v < C::LOADS_PER_G; ++v)
#pragma unroll
        for (int e = 0; e < C::VEC_IN; ++e) w[v * C::VEC_IN + e] = (float)rx[g][v][e];
      if (tail) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (k0 + kg + e >= K) w[e] = 0.0f;
      }
      *reinterpret_cast<f4_t*>(sx + row * LR + kg) = w;
    }
  };

  f4_t acc[FL][FP];
#pragma unroll
  for (int i = 0; i < FL; ++i)
#pragma unroll
    for (int j = 0; j < FP; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

  const int fr = lane & 15, fg = lane >> 4;
  auto compute_chunk = [&](int buf) {
    const float* sf = lds + buf * C::STAGE;
    const float* sx = sf + C::TILE_F;
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      float a[FL], b[FP];
#pragma unroll
      for (int i = 0; i < FL; ++i) a[i] = sf[(wm + 16 * i + fr) * LR + ks * 4 + fg];
#pragma unroll
      for (int j = 0; j < FP; ++j) b[j] = sx[(wn + 16 * j + fr) * LR + ks * 4 + fg];
#pragma unroll
      for (int i = 0; i < FL; ++i)
#pragma unroll
        for (int j = 0; j < FP; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  };

  load_chunk(0);
  store_chunk(0, 0);
  __syncthreads();
  for (int c = 0; c + 1 < nchunk; ++c) {
    load_chunk(c + 1);
    __builtin_amdgcn_sched_barrier(0);
    compute_chunk(c & 1);
    __builtin_amdgcn_sched_barrier(0);
    store_chunk((c + 1) & 1, c + 1);
    __syncthreads();
  }
  compute_chunk((nchunk - 1) & 1);

  // ---- epilogue: f32 16x16 layout: lane, reg r -> row 4*(lane/16) + r, col lane%16
  const EpiLP& epi = d.epi;
  int aidx[FP], bidx[FP];
  bool pok[FP];
#pragma unroll
  for (int j = 0; j < FP; ++j) {
    const long p = p0 + wn + 16 * j + fr;
    pok[j] = p < P;
    const int pi = (int)(pok[j] ? p : 0);
    aidx[j] = pi / B;
    bidx[j] = pi - aidx[j] * B;
  }
  double dmax = 0.0, umax = 0.0;
  double dab[FP];  // divide: l1[a] + l2[b] per column
#pragma unroll
  for (int j = 0; j < FP; ++j) dab[j] = EPI == EPI_DIVIDE ? epi.l1[aidx[j]] + epi.l2[bidx[j]] : 0.0;
#pragma unroll
  for (int i = 0; i < FL; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int l = l0 + wm + 16 * i + 4 * fg + r;
      if (l >= L) continue;
      const double dl = EPI == EPI_DIVIDE ? epi.l0[l] : 0.0;
#pragma unroll
      for (int j = 0; j < FP; ++j) {
        if (!pok[j]) continue;
        const size_t off = ((size_t)l * A + aidx[j]) * ldy + bidx[j];
        const float v = acc[i][j][r];
        if constexpr (EPI == EPI_STORE) {
          y[off] = (TOut)v;
        } else if constexpr (EPI == EPI_DIVIDE) {
          // the quotient is rounded to FP32 anyway: a fast float divide suffices
          y[off] = (TOut)__fdividef(v, (float)spectral_den(dl + dab[j], epi.alpha, epi.b1, epi.b2));
        } else {  // EPI_ACCUM into FP64 (TOut = double)
          const double dv = (double)v;
          const double un = epi.first ? dv : (double)y[off] + dv;
          y[off] = (TOut)un;
          // a NaN / Inf turns the norm into +Inf (fmax alone would drop NaN)
          dmax = fabs(dv) <= DBL_MAX ? fmax(dmax, fabs(dv)) : INFINITY;
          umax = fabs(un) <= DBL_MAX ? fmax(umax, fabs(un)) : INFINITY;
        }
      }
    }
  if constexpr (EPI == EPI_ACCUM) {
    if (epi.norms) {
      // wave max, then one atomic per wave on the bit pattern (non-negative
      // doubles order like their unsigned integer bits)
#pragma unroll
      for (int s = 32; s >= 1; s >>= 1) {
        dmax = fmax(dmax, __shfl_xor(dmax, s));
        umax = fmax(umax, __shfl_xor(umax, s));
      }
      if (lane == 0) {
        atomicMax(reinterpret_cast<unsigned long long*>(epi.norms), (unsigned long long)__double_as_longlong(dmax));
        atomicMax(reinterpret_cast<unsigned long long*>(epi.norms) + 1,
                  (unsigned long long)__double_as_longlong(umax));
      }
    }
  }
}

template <class TIn, class TT>
constexpr int lds_floats() {
  return 2 * Cfg<TIn, TT>::STAGE;
}

template <class TIn, class TOut, int EPI, class TT>
__global__ __launch_bounds__(TT::NTHREADS) void mode_rot_f32(LpDesc d, long ntiles, long nblocks_padded) {
  __shared__ __attribute__((aligned(16))) float lds[lds_floats<TIn, TT>()];
  const long t = xcd_tile(nblocks_padded);
  if (t >= ntiles) return;
  tile_body<TIn, TOut, EPI, TT>(d, t, lds);
}

// Persistent launch over the tiles of many passes: descriptor i owns tiles
// [tile0_i, tile0_i + tiles_i) of a global numbering; blocks stride over it.
// Descriptors of solves with active[sid] == 0 are skipped.
template <class TIn, class TOut, int EPI, class TT>
__global__ __launch_bounds__(TT::NTHREADS) void mode_rot_f32_batch(const LpDesc* __restrict__ descs, int nd,
                                                                   long total_tiles, const int* __restrict__ active) {
  __shared__ __attribute__((aligned(16))) float lds[lds_floats<TIn, TT>()];
  for (long i = blockIdx.x; i < total_tiles; i += gridDim.x) {
    int lo = 0, hi = nd;  // last descriptor with tile0 <= i
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (descs[mid].tile0 <= i) lo = mid;
      else hi = mid;
    }
    const LpDesc& d = descs[lo];
    if (!active[d.sid]) continue;  // uniform over the block, before any barrier of this tile
    tile_body<TIn, TOut, EPI, TT>(d, i - d.tile0, lds);
    __syncthreads();  // the next tile's first LDS store must not overtake this tile's reads
  }
}

template <class TIn, class TOut, int EPI, class TT>
hipError_t launch_single(const LpDesc& d0, hipStream_t stream) {
  LpDesc d = d0;
  d.tiles_l = (d.L + TT::BM - 1) / TT::BM;
  const long ntiles = (long)d.tiles_l * ((d.P + TT::BN - 1) / TT::BN);
  const long nbp = ((ntiles + 7) / 8) * 8;
  if (ntiles == 0) return hipSuccess;
  if (nbp > 0x7fffffffL) return hipErrorInvalidValue;
  mode_rot_f32<TIn, TOut, EPI, TT><<<dim3((unsigned)nbp), dim3(TT::NTHREADS), 0, stream>>>(d, ntiles, nbp);
  return hipGetLastError();
}

template <class TIn, class TOut, int EPI, class TT>
hipError_t launch_batch_t(const LpDesc* descs, int nd, long total_tiles, const int* active, int grid,
                          hipStream_t stream) {
  if (nd <= 0 || total_tiles <= 0) return hipSuccess;
  const long g = grid < total_tiles ? grid : total_tiles;
  mode_rot_f32_batch<TIn, TOut, EPI, TT><<<dim3((unsigned)g), dim3(TT::NTHREADS), 0, stream>>>(descs, nd,
                                                                                               total_tiles, active);
  return hipGetLastError();
}

template <class TIn, class TOut, int EPI>
hipError_t batch_by_tile(int tile_rows, const LpDesc* descs, int nd, long total_tiles, const int* active, int grid,
                         hipStream_t s) {
  switch (tile_rows) {
    case 128: return launch_batch_t<TIn, TOut, EPI, T128>(descs, nd, total_tiles, active, grid, s);
    case 96: return launch_batch_t<TIn, TOut, EPI, T96>(descs, nd, total_tiles, active, grid, s);
    case 64: return launch_batch_t<TIn, TOut, EPI, T64>(descs, nd, total_tiles, active, grid, s);
    case 32: return launch_batch_t<TIn, TOut, EPI, T32>(descs, nd, total_tiles, active, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace f32k

// ---------------------------------------------------------------------------
template <class TT>
static hipError_t launch_single_tile(const LpDesc& d, const LpPass& ps, hipStream_t stream) {
  using namespace f32k;
  if (ps.out_kind == 0)
    return ps.in_kind == 0 ? launch_single<double, double, EPI_ACCUM, TT>(d, stream)
                           : launch_single<float, double, EPI_ACCUM, TT>(d, stream);
  if (ps.epi_kind == EPI_DIVIDE)
    return ps.in_kind == 0 ? launch_single<double, float, EPI_DIVIDE, TT>(d, stream)
                           : launch_single<float, float, EPI_DIVIDE, TT>(d, stream);
  return ps.in_kind == 0 ? launch_single<double, float, EPI_STORE, TT>(d, stream)
                         : launch_single<float, float, EPI_STORE, TT>(d, stream);
}

bool lp_kind_ok(int in_kind, int out_kind, int epi) {
  if (out_kind == 0) return epi == EPI_ACCUM && (in_kind == 0 || in_kind == 1);
  return out_kind == 1 && epi != EPI_ACCUM && (in_kind == 0 || in_kind == 1);
}

hipError_t launch_mode_lp(const LpPass& ps, hipStream_t stream) {
  if (ps.mode != LP_F32 || !lp_kind_ok(ps.in_kind, ps.out_kind, ps.epi_kind)) return hipErrorInvalidValue;
  LpDesc d;
  d.x = ps.x;
  d.y = ps.y;
  d.f = ps.f_hi;
  d.epi = ps.epi;
  d.P = ps.P;
  d.ldx = ps.ldx;
  d.K = ps.K;
  d.ldy = ps.ldy;
  d.A = ps.A;
  d.B = ps.B;
  d.L = ps.L;
  d.ldf = ps.ldf;
  using namespace f32k;
  // a tuned tile shape, else 96-row factor tiles when they cover L with clearly
  // fewer padded rows (e.g. L = 257: 288 rows instead of 384)
  switch (ps.tile_rows) {
    case 128: return launch_single_tile<T128>(d, ps, stream);
    case 96: return launch_single_tile<T96>(d, ps, stream);
    case 64: return launch_single_tile<T64>(d, ps, stream);
    case 32: return launch_single_tile<T32>(d, ps, stream);
    default: break;
  }
  const long r128 = (ps.L + 127) / 128 * 128, r96 = (ps.L + 95) / 96 * 96;
  if (r96 * 10 < r128 * 9) return launch_single_tile<T96>(d, ps, stream);
  return launch_single_tile<T128>(d, ps, stream);
}

hipError_t launch_mode_f32_batch(int in_kind, int out_kind, int epi, int tile_rows, const LpDesc* descs, int nd,
                                 long total_tiles, const int* active, int grid, hipStream_t stream) {
  if (!lp_kind_ok(in_kind, out_kind, epi)) return hipErrorInvalidValue;
  using namespace f32k;
  if (out_kind == 0)
    return in_kind == 0 ? batch_by_tile<double, double, EPI_ACCUM>(tile_rows, descs, nd, total_tiles, active, grid,
                                                                   stream)
                        : batch_by_tile<float, double, EPI_ACCUM>(tile_rows, descs, nd, total_tiles, active, grid,
                                                                  stream);
  if (epi == EPI_DIVIDE)
    return in_kind == 0 ? batch_by_tile<double, float, EPI_DIVIDE>(tile_rows, descs, nd, total_tiles, active, grid,
                                                                   stream)
                        : batch_by_tile<float, float, EPI_DIVIDE>(tile_rows, descs, nd, total_tiles, active, grid,
                                                                  stream);
  return in_kind == 0
             ? batch_by_tile<double, float, EPI_STORE>(tile_rows, descs, nd, total_tiles, active, grid, stream)
             : batch_by_tile<float, float, EPI_STORE>(tile_rows, descs, nd, total_tiles, active, grid, stream);
}

int lp_batch_blocks_per_cu(int tile_rows) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  using namespace f32k;
  switch (tile_rows) {
    case 128:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, mode_rot_f32_batch<float, float, EPI_STORE, T128>,
                                                       T128::NTHREADS, 0);
      break;
    case 96:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, mode_rot_f32_batch<float, float, EPI_STORE, T96>,
                                                       T96::NTHREADS, 0);
      break;
    case 64:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, mode_rot_f32_batch<float, float, EPI_STORE, T64>,
                                                       T64::NTHREADS, 0);
      break;
    case 32:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, mode_rot_f32_batch<float, float, EPI_STORE, T32>,
                                                       T32::NTHREADS, 0);
      break;
    default:
      break;
  }
  return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace semfd
