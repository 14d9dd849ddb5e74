// Low-precision mode products (FP32 MFMA, BF16 MFMA, split BF16) for the
// mixed-precision refinement path.
//
// Each pass contracts the CONTIGUOUS axis of its input and writes the output
// with the axes rotated:  X (A, B, K) -> Y (K', A, B),
//        Y[l][a][b] = sum_k F[l][k] X[a][b][k].
// Three passes rotate (x, y, z) -> (z, x, y) -> (y, z, x) -> (x, y, z), so the
// three forward products (and the three backward ones) of eq. 3D-Poisson return
// to the caller's layout while every pass reads both MFMA operands -- factor
// rows F[l][:] and tensor rows X[p][:] -- contiguously along the contraction.
// No transposes are needed, which matters for the BF16 MFMA whose fragments
// hold 8 consecutive contraction elements per lane.
//
// GEMM view:  C[l][p] = sum_k F[l][k] X[p][k],  p = a*B + b, output address
// (l*A + a)*ldy + b.  Block tile 128 (l) x 128 (p), 4 waves of 64 x 64.
//
// Precision modes:
//   LP_F32    : FP32 operands, v_mfma_f32_16x16x4_f32.
//   LP_BF16   : BF16 operands, v_mfma_f32_16x16x32_bf16, FP32 accumulation.
//   LP_BF16X3 : operands split as hi + lo BF16 (hi = bf16(v), lo = bf16(v - hi));
//               three MFMAs per step (hi*hi + hi*lo + lo*hi), FP32 accumulation.
// Epilogues: store (BF16 / FP32 intermediates), eigenvalue divide (third
// forward pass), or accumulate into the FP64 solution (u += delta) while
// recording max|delta| and max|u| for the refinement stop test.
#include <hip/hip_runtime.h>

#include <cfloat>

#include <cstdint>

#include "kernels.h"

namespace semfd {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef unsigned short us8_t __attribute__((ext_vector_type(8)));

namespace lpk {

// Block tile BM (l) x BN (p) on WL x WP waves; each wave owns a (BM/WL) x (BN/WP)
// sub-tile of 16 x 16 MFMA tiles.
template <int BM_, int BN_, int WL_, int WP_>
struct Tile {
  static constexpr int BM = BM_, BN = BN_, WL = WL_, WP = WP_;
  static constexpr int NTHREADS = 64 * WL * WP;
  static constexpr int TL = BM / WL, TP = BN / WP;  // wave tile
  static constexpr int FL = TL / 16, FP = TP / 16;  // MFMA tiles per wave
};
typedef Tile<128, 128, 2, 2> TileS;  // 4 waves, 64 x 64 per wave
typedef Tile<256, 256, 2, 4> TileL;  // 8 waves, 128 x 64 per wave

// float -> bf16 bits, round to nearest even (NaN kept quiet)
__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float(((unsigned)b) << 16); }

template <class T>
__device__ __forceinline__ float to_f(T v);
template <>
__device__ __forceinline__ float to_f<float>(float v) { return v; }
template <>
__device__ __forceinline__ float to_f<double>(double v) { return (float)v; }
template <>
__device__ __forceinline__ float to_f<unsigned short>(unsigned short v) { return bf2f(v); }

__device__ __forceinline__ long xcd_tile(long nblocks_padded) {
  const long per = nblocks_padded / 8;
  return (long)(blockIdx.x % 8) * per + (long)(blockIdx.x / 8);
}

// Operand element type in LDS: float for LP_F32, bf16 bits otherwise.
template <int MODE>
struct OpT {
  typedef unsigned short type;
};
template <>
struct OpT<LP_F32> {
  typedef float type;
};

// BK (contraction chunk): 32 for FP32 (8 MFMA steps of 4), for FP64 input
// (register budget) and for split BF16 (four LDS tiles); 64 otherwise (2 BF16
// MFMA steps of 32).
template <int MODE, class TIn, class TT>
struct Cfg {
  static constexpr int BM = TT::BM, BN = TT::BN, NTHREADS = TT::NTHREADS;
  static constexpr int BK = (MODE == LP_F32 || MODE == LP_BF16X3 || sizeof(TIn) == 8) ? 32 : 64;
  typedef typename OpT<MODE>::type op_t;
  static constexpr int PAD = 16 / (int)sizeof(op_t);      // 16 bytes of row padding
  static constexpr int LDS_ROW = BK + PAD;                 // elements per LDS row
  static constexpr int NSPLIT = MODE == LP_BF16X3 ? 2 : 1;  // hi (+ lo) copies
  static_assert(BM == BN, "factor and tensor tiles share one row count");
  static constexpr int TILE = BM * LDS_ROW;                 // elements per [BM][BK] tile
  // tensor staging: each thread handles groups of G consecutive contraction
  // elements (16 bytes of operand type); a group is read with 16-byte vector
  // loads, or 8-byte loads for FP64 input (whose rows may be odd-sized).
  static constexpr int G = 16 / (int)sizeof(op_t);
  static constexpr int VEC_IN = sizeof(TIn) == 8 ? 1 : 16 / (int)sizeof(TIn);
  static constexpr int LOADS_PER_G = G / VEC_IN;
  static constexpr int NGROUP = BM * BK / G / NTHREADS;
  // factor loads: 16-byte vectors of op_t
  static constexpr int VEC_F = 16 / (int)sizeof(op_t);
  static constexpr int NLOAD_F = BM * BK / VEC_F / NTHREADS;
};

template <int MODE, class TIn, class TOut, int EPI, class TT>
__global__ __launch_bounds__(TT::NTHREADS) void mode_rot_lp(const TIn* __restrict__ x, int ldx, long P, int K,
                                                           TOut* __restrict__ y, int ldy, int A, int B, int L,
                                                           const void* __restrict__ f_hi,
                                                           const void* __restrict__ f_lo, int ldf, long tiles_l,
                                                           long ntiles, long nblocks_padded, EpiLP epi) {
  typedef Cfg<MODE, TIn, TT> C;
  typedef typename C::op_t op_t;
  constexpr int BK = C::BK, LR = C::LDS_ROW, NS = C::NSPLIT;
  constexpr int BM = TT::BM, BN = TT::BN, NTHREADS = TT::NTHREADS, FL = TT::FL, FP = TT::FP;
  // per stage: NS factor tiles + NS tensor tiles
  __shared__ __attribute__((aligned(16))) op_t lds[2 * 2 * NS * C::TILE];

  const long t = xcd_tile(nblocks_padded);
  if (t >= ntiles) return;
  const long lt = t % tiles_l;
  const long pt = t / tiles_l;
  const int l0 = (int)(lt * BM);
  const long p0 = pt * BN;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / TT::WP) * TT::TL;  // rows: l
  const int wn = (wave % TT::WP) * TT::TP;  // cols: p

  // ---- global load mapping -------------------------------------------------
  // Consecutive lanes take consecutive groups of one row, so loads are contiguous.
  constexpr int G_PER_ROW = BK / C::G;
  constexpr int FV_PER_ROW = BK / C::VEC_F;
  const TIn* __restrict__ xb = x + (size_t)p0 * ldx;
  const int prow_max = (int)(P - 1 - p0);

  typedef TIn xvec_t __attribute__((ext_vector_type(C::VEC_IN)));
  xvec_t rx[C::NGROUP][C::LOADS_PER_G];
  us8_t rf_hi[C::NLOAD_F];  // 16 bytes each, reinterpreted per mode
  us8_t rf_lo[NS == 2 ? C::NLOAD_F : 1];
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
      const int kk = (idx % FV_PER_ROW) * C::VEC_F;
      const size_t off = (size_t)(l0 + row) * ldf + k0 + kk;  // factor padded: always in bounds
      rf_hi[v] = *reinterpret_cast<const us8_t*>(reinterpret_cast<const op_t*>(f_hi) + off);
      if constexpr (NS == 2) rf_lo[v] = *reinterpret_cast<const us8_t*>(reinterpret_cast<const op_t*>(f_lo) + off);
    }
  };

  auto store_chunk = [&](int buf, int c) {
    op_t* sbase = lds + buf * (2 * NS * C::TILE);
    op_t* sf_hi = sbase;
    op_t* sf_lo = sbase + C::TILE;
    op_t* sx_hi = sbase + NS * C::TILE;
    op_t* sx_lo = sbase + NS * C::TILE + C::TILE;
    const int k0 = c * BK;
    const bool tail = k0 + BK > K;  // uniform: only the last chunk
#pragma unroll
    for (int v = 0; v < C::NLOAD_F; ++v) {
      const int idx = v * NTHREADS + tid;
      const int row = idx / FV_PER_ROW;
      const int kk = (idx % FV_PER_ROW) * C::VEC_F;
      *reinterpret_cast<us8_t*>(sf_hi + row * LR + kk) = rf_hi[v];
      if constexpr (NS == 2) *reinterpret_cast<us8_t*>(sf_lo + row * LR + kk) = rf_lo[v];
    }
    constexpr bool passthrough = NS == 1 && sizeof(TIn) == sizeof(op_t);
#pragma unroll
    for (int g = 0; g < C::NGROUP; ++g) {
      const int idx = g * NTHREADS + tid;
      const int row = idx / G_PER_ROW;
      const int kg = (idx % G_PER_ROW) * C::G;
      if constexpr (passthrough) {
        // same element type in HBM and LDS: store the loaded 16 bytes as they are
        xvec_t v = rx[g][0];
        if (tail) {
#pragma unroll
          for (int e = 0; e < C::G; ++e)
            if (k0 + kg + e >= K) v[e] = (TIn)0;
        }
        *reinterpret_cast<xvec_t*>(sx_hi + row * LR + kg) = v;
        continue;
      }
      // gather the group as floats and convert
      float fv[C::G];
#pragma unroll
      for (int v = 0; v < C::LOADS_PER_G; ++v)
#pragma unroll
        for (int e = 0; e < C::VEC_IN; ++e) fv[v * C::VEC_IN + e] = to_f<TIn>(rx[g][v][e]);
      if (tail) {
#pragma unroll
        for (int e = 0; e < C::G; ++e)
          if (k0 + kg + e >= K) fv[e] = 0.0f;
      }
      if constexpr (MODE == LP_F32) {
        f4_t w = {fv[0], fv[1], fv[2], fv[3]};
        *reinterpret_cast<f4_t*>(sx_hi + row * LR + kg) = w;
      } else {
        bf8_t h, lo;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          h[e] = (__bf16)fv[e];
          if constexpr (NS == 2) lo[e] = (__bf16)(fv[e] - (float)h[e]);
        }
        *reinterpret_cast<bf8_t*>(sx_hi + row * LR + kg) = h;
        if constexpr (NS == 2) *reinterpret_cast<bf8_t*>(sx_lo + row * LR + kg) = lo;
      }
    }
  };

  f4_t acc[FL][FP];
#pragma unroll
  for (int i = 0; i < FL; ++i)
#pragma unroll
    for (int j = 0; j < FP; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

  const int fr = lane & 15, fg = lane >> 4;
  auto compute_chunk = [&](int buf) {
    const op_t* sbase = lds + buf * (2 * NS * C::TILE);
    const op_t* sf_hi = sbase;
    const op_t* sf_lo = sbase + C::TILE;
    const op_t* sx_hi = sbase + NS * C::TILE;
    const op_t* sx_lo = sbase + NS * C::TILE + C::TILE;
    if constexpr (MODE == LP_F32) {
#pragma unroll
      for (int ks = 0; ks < BK / 4; ++ks) {
        float a[FL], b[FP];
#pragma unroll
        for (int i = 0; i < FL; ++i) a[i] = sf_hi[(wm + 16 * i + fr) * LR + ks * 4 + fg];
#pragma unroll
        for (int j = 0; j < FP; ++j) b[j] = sx_hi[(wn + 16 * j + fr) * LR + ks * 4 + fg];
#pragma unroll
        for (int i = 0; i < FL; ++i)
#pragma unroll
          for (int j = 0; j < FP; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < BK / 32; ++ks) {
        bf8_t a[FL], b[FP], alo[NS == 2 ? FL : 1], blo[NS == 2 ? FP : 1];
#pragma unroll
        for (int i = 0; i < FL; ++i) {
          const int off = (wm + 16 * i + fr) * LR + ks * 32 + 8 * fg;
          a[i] = *reinterpret_cast<const bf8_t*>(sf_hi + off);
          if constexpr (NS == 2) alo[i] = *reinterpret_cast<const bf8_t*>(sf_lo + off);
        }
#pragma unroll
        for (int j = 0; j < FP; ++j) {
          const int off = (wn + 16 * j + fr) * LR + ks * 32 + 8 * fg;
          b[j] = *reinterpret_cast<const bf8_t*>(sx_hi + off);
          if constexpr (NS == 2) blo[j] = *reinterpret_cast<const bf8_t*>(sx_lo + off);
        }
#pragma unroll
        for (int i = 0; i < FL; ++i)
#pragma unroll
          for (int j = 0; j < FP; ++j) {
            if constexpr (NS == 2) {
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[i], b[j], acc[i][j], 0, 0, 0);
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], blo[j], acc[i][j], 0, 0, 0);
            }
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
          }
      }
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
        if constexpr (EPI == EPI_STORE || EPI == EPI_DIVIDE) {
          float w = v;
          // the quotient is rounded to FP32 / BF16 anyway: a fast float divide suffices
          if constexpr (EPI == EPI_DIVIDE) w = __fdividef(v, (float)spectral_den(dl + dab[j], epi.alpha, epi.b1, epi.b2));
          if constexpr (sizeof(TOut) == 2)
            y[off] = __builtin_bit_cast(unsigned short, (__bf16)w);
          else
            y[off] = (TOut)w;
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
      // doubles order like their unsigned integer bits; NaN sorts above Inf)
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

}  // namespace lpk

// ---------------------------------------------------------------------------
template <int MODE, class TIn, class TOut, int EPI, class TT>
static hipError_t launch_tile(const LpPass& ps, hipStream_t stream) {
  using namespace lpk;
  const long tiles_l = (ps.L + TT::BM - 1) / TT::BM;
  const long tiles_p = (ps.P + TT::BN - 1) / TT::BN;
  const long ntiles = tiles_l * tiles_p;
  const long nbp = ((ntiles + 7) / 8) * 8;
  if (nbp > 0x7fffffffL || ntiles == 0) return ntiles == 0 ? hipSuccess : hipErrorInvalidValue;
  mode_rot_lp<MODE, TIn, TOut, EPI, TT><<<dim3((unsigned)nbp), dim3(TT::NTHREADS), 0, stream>>>(
      (const TIn*)ps.x, ps.ldx, ps.P, ps.K, (TOut*)ps.y, ps.ldy, ps.A, ps.B, ps.L, ps.f_hi, ps.f_lo, ps.ldf, tiles_l,
      ntiles, nbp, ps.epi);
  return hipGetLastError();
}

// The 256 x 256 tile halves the L2 traffic per flop of the BF16 modes (whose
// passes are bound by it); it is used when padding the factor rows to 256 costs
// no more than ~8 % extra work and the tensor has enough rows to fill the chip.
// The FP32 mode is MFMA-bound and keeps the 128 x 128 tile.
template <int MODE, class TIn, class TOut, int EPI>
static hipError_t launch_one(const LpPass& ps, hipStream_t stream) {
  const long pad256 = (ps.L + 255) / 256 * 256;
  if (MODE != LP_F32 && ps.P >= 65536 && pad256 * 100 <= (long)ps.L * 108 && ps.ldf >= pad256)
    return launch_tile<MODE, TIn, TOut, EPI, lpk::TileL>(ps, stream);
  return launch_tile<MODE, TIn, TOut, EPI, lpk::TileS>(ps, stream);
}

// in_kind: 0 = FP64, 1 = FP32, 2 = BF16 (bits);  out_kind: 1 = FP32, 2 = BF16, 0 = FP64 accumulate
template <int MODE>
static hipError_t dispatch_mode(const LpPass& ps, hipStream_t s) {
  typedef unsigned short bf;
  const int ik = ps.in_kind, ok = ps.out_kind, ep = ps.epi_kind;
  if (ok == 0) {  // accumulate into FP64
    if (ep != EPI_ACCUM) return hipErrorInvalidValue;
    if (ik == 1) return launch_one<MODE, float, double, EPI_ACCUM>(ps, s);
    if (ik == 2) return launch_one<MODE, bf, double, EPI_ACCUM>(ps, s);
    if (ik == 0) return launch_one<MODE, double, double, EPI_ACCUM>(ps, s);
    return hipErrorInvalidValue;
  }
  if (ep == EPI_ACCUM) return hipErrorInvalidValue;
#define SEMFD_LP_CASE(TI, TO)                                                          \
  return ep == EPI_DIVIDE ? launch_one<MODE, TI, TO, EPI_DIVIDE>(ps, s)                \
                          : launch_one<MODE, TI, TO, EPI_STORE>(ps, s)
  if (ik == 0 && ok == 1) SEMFD_LP_CASE(double, float);
  if (ik == 0 && ok == 2) SEMFD_LP_CASE(double, bf);
  if (ik == 1 && ok == 1) SEMFD_LP_CASE(float, float);
  if (ik == 1 && ok == 2) SEMFD_LP_CASE(float, bf);
  if (ik == 2 && ok == 2) SEMFD_LP_CASE(bf, bf);
  if (ik == 2 && ok == 1) SEMFD_LP_CASE(bf, float);
#undef SEMFD_LP_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_mode_lp(const LpPass& ps, hipStream_t stream) {
  switch (ps.mode) {
    case LP_F32:
      return dispatch_mode<LP_F32>(ps, stream);
    case LP_BF16:
      return dispatch_mode<LP_BF16>(ps, stream);
    case LP_BF16X3:
      return dispatch_mode<LP_BF16X3>(ps, stream);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace semfd
