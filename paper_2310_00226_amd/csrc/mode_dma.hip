// BF16 rotating mode products with direct global -> LDS loads.
//
// Same contraction as the FP32 passes (Y[l][a][b] = sum_k F[l][k] X[a][b][k],
// the axes rotating from pass to pass) for the two BF16 modes, organised for
// CDNA4:
//  * operand tiles move from HBM / L2 straight into LDS with
//    global_load_lds_dwordx4 (no VGPR staging), through a ring of STAGES buffers
//    addressed with compile-time indices (the chunk loop is unrolled by STAGES);
//    the kernel orders DMA and LDS reads itself (vmcnt waits + barriers);
//  * LDS rows are 64 bytes (32 BF16 = one 16x16x32 MFMA step) made of four
//    16-byte chunks placed at slot chunk ^ g(row), g(row) = ((row>>1)^(row>>2))&3,
//    which makes the fragment reads (16 rows x one chunk per 16 lanes)
//    bank-conflict-free for 32 and 64 four-byte banks;
//  * ping-pong wave groups: the 8 waves of a block form two groups of 4, one
//    wave of each per SIMD.  While one group issues MFMAs the other issues the
//    DMA and reads its next fragments from LDS; block barriers switch the roles
//    twice per chunk, so every SIMD's MFMA unit is fed by one wave while its
//    partner waits on memory;
//  * block tile BML (l) x 256 (p): BF16 256 x 256 with waves of 128 x 64;
//    split BF16 (three MFMAs per step, twice the operands) 128 x 256 with waves
//    of 64 x 64 to stay within the register file.
// Split BF16 (LP_BF16X3) keeps every operand as two BF16 planes (hi, lo) in
// HBM, so its intermediates load without conversion too.
//
// Contract of the operands (set up by the caller):
//  * tensor rows have a pitch ldx that is a multiple of 8 elements (16 bytes);
//    elements between K and ldx hold finite values (they meet zero factor
//    columns), and the second plane (split mode) starts xplane elements after
//    the first;
//  * the factor is [l][k] with pitch ldf (multiple of 8, >= 256-rounded L and
//    32-rounded K), zero outside L x K, second plane fplane elements after the first.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdint>

#include "kernels.h"

namespace semfd {

namespace dmak {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void lds_void;

constexpr int NTHREADS = 512;  // 8 waves
constexpr int BN = 256;        // tensor rows per block tile
constexpr int TP = 64;         // tensor rows per wave
constexpr int FP = TP / 16;    // 4 MFMA tiles along p
constexpr int BK = 32;         // BF16 elements per chunk (64-byte LDS rows)
constexpr int ROWB = BK * 2;   // bytes per LDS row

__device__ __forceinline__ int swz(int row) { return ((row >> 1) ^ (row >> 2)) & 3; }

__device__ __forceinline__ long xcd_tile(long nblocks_padded) {
  const long per = nblocks_padded / 8;
  return (long)(blockIdx.x % 8) * per + (long)(blockIdx.x / 8);
}

// s_waitcnt vmcnt(N) lgkmcnt(0) (expcnt untouched), gfx9 encoding
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (0 << 8) | ((N >> 4) << 14));
}

template <int MODE>
struct KCfg {
  static constexpr int NS = MODE == LP_BF16X3 ? 2 : 1;  // operand planes
  static constexpr int BML = NS == 2 ? 128 : 256;      // factor rows per block tile
  static constexpr int TL = BML / 2;                   // factor rows per wave (two groups)
  static constexpr int FL = TL / 16;
  static constexpr int TILEF = BML * ROWB;             // bytes of one factor tile plane
  static constexpr int TILEX = BN * ROWB;              // bytes of one tensor tile plane
  static constexpr int PLANEB = TILEF + TILEX;
  static constexpr int STAGEB = NS * PLANEB;
  static constexpr int STAGES = NS == 2 ? 3 : 4;       // 144 KB / 128 KB of LDS
  // DMA instructions per chunk per wave of group 0 (16 rows of 64 bytes each)
  static constexpr int FQ = BML / 16 / 4, XQ = BN / 16 / 4;
  static constexpr int D = NS * (FQ + XQ);
  static_assert((STAGES - 2) * D < 64, "vmcnt range");
};

template <int MODE, class TOut, int EPI>
__global__ __launch_bounds__(NTHREADS) void mode_rot_dma(const unsigned short* __restrict__ x, int ldx, long xplane,
                                                         long P, int K, TOut* __restrict__ y, int ldy, long yplane,
                                                         int A, int B, int L, const unsigned short* __restrict__ f,
                                                         int ldf, long fplane, long tiles_l, long ntiles,
                                                         long nblocks_padded, EpiLP epi) {
  typedef KCfg<MODE> C;
  constexpr int NS = C::NS, S = C::STAGES, FL = C::FL;
  __shared__ __attribute__((aligned(1024))) unsigned char ring[S][C::STAGEB];

  const long t = xcd_tile(nblocks_padded);
  if (t >= ntiles) return;  // whole block leaves together, before any barrier
  const long lt = t % tiles_l;
  const long pt = t / tiles_l;
  const int l0 = (int)(lt * C::BML);
  const long p0 = pt * BN;

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // Waves w and w + 4 share SIMD w % 4.  Group 0 (waves 0-3) owns factor rows
  // 0 .. TL-1 of the tile, group 1 (waves 4-7) rows TL .. 2 TL-1; within a group
  // wave w % 4 owns tensor rows 64 (w % 4) .. + 63.
  const bool g0 = wave < 4;
  const int gw = wave & 3;
  const int wm = g0 ? 0 : C::TL;
  const int wn = gw * TP;
  const int nchunk = (K + BK - 1) / BK;

  // ---- DMA (group 0 only) ----------------------------------------------------
  // One instruction fills 16 LDS rows: lane i writes slot i % 4 of row
  // row0 + i / 4 and therefore fetches chunk (i % 4) ^ g(row) of that row.  Wave
  // gw fills factor rows [FQ*16*gw, +FQ*16) and tensor rows [XQ*16*gw, +XQ*16).
  // Addresses are a wave-uniform base plus a 32-bit per-lane offset.
  auto issue = [&](unsigned char* stage, int c) {
    const int k0 = c * BK;
#pragma unroll
    for (int q = 0; q < C::FQ; ++q) {  // factor: padded to whole tiles, always in bounds
      const int rowq = 16 * (C::FQ * gw + q);
      const int row = rowq + lane / 4;
      const int kc = ((lane & 3) ^ swz(row)) * 8;
      const unsigned short* fb = f + (size_t)(l0 + rowq) * ldf + k0;
      const unsigned foff = (unsigned)((lane / 4) * ldf + kc);
#pragma unroll
      for (int pl = 0; pl < NS; ++pl)
        __builtin_amdgcn_global_load_lds((const void*)(fb + pl * fplane + foff),
                                         (lds_void*)(stage + pl * C::PLANEB + rowq * ROWB), 16, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < C::XQ; ++q) {
      // tensor: rows past P read row P - 1; chunks past the row pitch read the
      // row start (finite data times zero factor columns)
      const int rowq = 16 * (C::XQ * gw + q);
      const int row = rowq + lane / 4;
      const int kc = ((lane & 3) ^ swz(row)) * 8;
      const long rq = p0 + rowq < P ? p0 + rowq : P - 1;
      const long rl = p0 + row < P ? p0 + row : P - 1;
      const unsigned short* xb = x + (size_t)rq * ldx;
      const int kx = k0 + kc < ldx ? k0 + kc : 0;
      const unsigned xoff = (unsigned)((rl - rq) * ldx + kx);
#pragma unroll
      for (int pl = 0; pl < NS; ++pl)
        __builtin_amdgcn_global_load_lds((const void*)(xb + pl * xplane + xoff),
                                         (lds_void*)(stage + pl * C::PLANEB + C::TILEF + rowq * ROWB), 16, 0, 0);
    }
  };

  f4_t acc[FL][FP];
#pragma unroll
  for (int i = 0; i < FL; ++i)
#pragma unroll
    for (int j = 0; j < FP; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

  const int fr = lane & 15, fg = lane >> 4;
  // fragment byte offsets within a stage (row-dependent swizzle)
  int aoff[FL], boff[FP];
#pragma unroll
  for (int i = 0; i < FL; ++i) {
    const int row = wm + 16 * i + fr;
    aoff[i] = row * ROWB + ((fg ^ swz(row)) << 4);
  }
#pragma unroll
  for (int j = 0; j < FP; ++j) {
    const int row = wn + 16 * j + fr;
    boff[j] = C::TILEF + row * ROWB + ((fg ^ swz(row)) << 4);
  }
  bf8_t a[FL], b[FP], alo[NS == 2 ? FL : 1], blo[NS == 2 ? FP : 1];
  auto read_frags = [&](const unsigned char* stage) {
#pragma unroll
    for (int i = 0; i < FL; ++i) a[i] = *reinterpret_cast<const bf8_t*>(stage + aoff[i]);
#pragma unroll
    for (int j = 0; j < FP; ++j) b[j] = *reinterpret_cast<const bf8_t*>(stage + boff[j]);
    if constexpr (NS == 2) {
#pragma unroll
      for (int i = 0; i < FL; ++i) alo[i] = *reinterpret_cast<const bf8_t*>(stage + C::PLANEB + aoff[i]);
#pragma unroll
      for (int j = 0; j < FP; ++j) blo[j] = *reinterpret_cast<const bf8_t*>(stage + C::PLANEB + boff[j]);
    }
  };
  // products outermost: consecutive MFMAs write different accumulators
  auto mfmas = [&]() {
    if constexpr (NS == 2) {
#pragma unroll
      for (int i = 0; i < FL; ++i)
#pragma unroll
        for (int j = 0; j < FP; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[i], b[j], acc[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < FL; ++i)
#pragma unroll
        for (int j = 0; j < FP; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], blo[j], acc[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < FL; ++i)
#pragma unroll
      for (int j = 0; j < FP; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  };
  // a phase boundary: nothing moves across it
  auto phase_end = [&]() {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
  };

  // ---- ping-pong pipeline ---------------------------------------------------------
  // Chunk c is handled in two phases separated by block barriers:
  //   phase 2c   : group 0 issues the DMA of chunk c + S - 1 and reads its chunk-c
  //                fragments; group 1 multiplies chunk c - 1;
  //   phase 2c+1 : group 0 multiplies chunk c; group 1 reads its chunk-c fragments.
  // Only group 0 issues DMA, exactly D instructions per chunk (past the last
  // chunk it reloads the last chunk into the free stage, never read), so one
  // constant vmcnt wait at the end of phase 2c+1 guarantees its part of chunk
  // c + 1; the following barrier publishes every wave's part.  The stage refilled
  // in phase 2c held chunk c - 1, read by group 1 in phase 2c - 1 (which waits for
  // its reads before that phase ends).  Both groups pass 1 + 2 nchunk barriers.
  const int clast = nchunk - 1;
  if (g0) {
#pragma unroll
    for (int s = 0; s + 1 < S; ++s) issue(ring[s], s < clast ? s : clast);
    wait_vm<(S - 2) * C::D>();
    phase_end();
    for (int c = 0; c < nchunk; c += S) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        if (c + s < nchunk) {
          const int cn = c + s + S - 1;
          issue(ring[(s + S - 1) % S], cn < clast ? cn : clast);
          read_frags(ring[s]);
          phase_end();
          mfmas();
          wait_vm<(S - 2) * C::D>();  // this wave's DMA of chunk c + s + 1 landed
          phase_end();
        }
      }
    }
    wait_vm<0>();  // drain the trailing reloads before the LDS is released
  } else {
    phase_end();
    for (int c = 0; c < nchunk; c += S) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        if (c + s < nchunk) {
          if (c + s > 0) mfmas();
          phase_end();
          read_frags(ring[s]);
          wait_vm<63>();  // lgkmcnt(0): fragments in registers before the stage can be refilled
          phase_end();
        }
      }
    }
    mfmas();  // the last chunk (group 0 is already in its epilogue)
  }

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
  double dab[FP];
#pragma unroll
  for (int j = 0; j < FP; ++j) dab[j] = EPI == EPI_DIVIDE ? epi.l1[aidx[j]] + epi.l2[bidx[j]] : 0.0;
  double dmax = 0.0, umax = 0.0;
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
        const size_t rowb = ((size_t)l * A + aidx[j]) * ldy;
        const size_t off = rowb + bidx[j];
        const float v = acc[i][j][r];
        if constexpr (EPI == EPI_ACCUM) {
          const double dv = (double)v;
          const double un = epi.first ? dv : (double)y[off] + dv;
          y[off] = (TOut)un;
          // a NaN / Inf turns the norm into +Inf (fmax alone would drop NaN)
          dmax = fabs(dv) <= DBL_MAX ? fmax(dmax, fabs(dv)) : INFINITY;
          umax = fabs(un) <= DBL_MAX ? fmax(umax, fabs(un)) : INFINITY;
        } else {
          float w = v;
          if constexpr (EPI == EPI_DIVIDE)
            w = __fdividef(v, (float)spectral_den(dl + dab[j], epi.alpha, epi.b1, epi.b2));
          const __bf16 h = (__bf16)w;
          y[off] = __builtin_bit_cast(unsigned short, h);
          if constexpr (NS == 2) y[off + yplane] = __builtin_bit_cast(unsigned short, (__bf16)(w - (float)h));
          // the row's last element also clears the pitch padding that the next
          // pass reads (against zero factor columns)
          if (bidx[j] == B - 1) {
            for (int e = B; e < ldy; ++e) {
              y[rowb + e] = 0;
              if constexpr (NS == 2) y[rowb + e + yplane] = 0;
            }
          }
        }
      }
    }
  if constexpr (EPI == EPI_ACCUM) {
    if (epi.norms) {
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

// FP64 caller-layout array (pitch nz) -> BF16 (hi [+ lo] planes) with pitch ldo,
// padding zeroed.  One wave per row.
template <int NS>
__global__ __launch_bounds__(256) void to_lowp_kernel(const double* __restrict__ f, unsigned short* __restrict__ o,
                                                      long plane_o, long rows, int nz, int ldo) {
  const long row = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  for (int e = (int)(threadIdx.x & 63); e < ldo; e += 64) {
    const float v = e < nz ? (float)f[(size_t)row * nz + e] : 0.0f;
    const __bf16 h = (__bf16)v;
    o[(size_t)row * ldo + e] = __builtin_bit_cast(unsigned short, h);
    if (NS == 2) o[(size_t)row * ldo + e + plane_o] = __builtin_bit_cast(unsigned short, (__bf16)(v - (float)h));
  }
}

}  // namespace dmak

bool dma_supported(const LpPass& ps) {
  // whole 256-row factor tiles must exist in the padded factor; the tensor pitch
  // must keep 16-byte chunks aligned
  const long pad256 = (ps.L + 255) / 256 * 256;
  return (ps.mode == LP_BF16 || ps.mode == LP_BF16X3) && ps.in_kind == 2 && ps.ldf >= pad256 &&
         ps.ldf % 8 == 0 && ps.ldx % 8 == 0 && ps.ldx >= ps.K && ps.ldf >= (ps.K + 31) / 32 * 32;
}

template <int MODE, class TOut, int EPI>
static hipError_t launch_dma_t(const LpPass& ps, hipStream_t stream) {
  using namespace dmak;
  constexpr int BML = KCfg<MODE>::BML;
  const long tiles_l = (ps.L + BML - 1) / BML;
  const long tiles_p = (ps.P + BN - 1) / BN;
  const long ntiles = tiles_l * tiles_p;
  const long nbp = ((ntiles + 7) / 8) * 8;
  if (ntiles == 0) return hipSuccess;
  if (nbp > 0x7fffffffL) return hipErrorInvalidValue;
  mode_rot_dma<MODE, TOut, EPI><<<dim3((unsigned)nbp), dim3(NTHREADS), 0, stream>>>(
      (const unsigned short*)ps.x, ps.ldx, ps.xplane, ps.P, ps.K, (TOut*)ps.y, ps.ldy, ps.yplane, ps.A, ps.B, ps.L,
      (const unsigned short*)ps.f_hi, ps.ldf, ps.fplane, tiles_l, ntiles, nbp, ps.epi);
  return hipGetLastError();
}

template <int MODE>
static hipError_t dispatch_dma(const LpPass& ps, hipStream_t s) {
  if (ps.out_kind == 0) {
    if (ps.epi_kind != EPI_ACCUM) return hipErrorInvalidValue;
    return launch_dma_t<MODE, double, EPI_ACCUM>(ps, s);
  }
  if (ps.out_kind != 2) return hipErrorInvalidValue;
  if (ps.epi_kind == EPI_DIVIDE) return launch_dma_t<MODE, unsigned short, EPI_DIVIDE>(ps, s);
  if (ps.epi_kind == EPI_STORE) return launch_dma_t<MODE, unsigned short, EPI_STORE>(ps, s);
  return hipErrorInvalidValue;
}

hipError_t launch_mode_dma(const LpPass& ps, hipStream_t stream) {
  if (!dma_supported(ps)) return hipErrorInvalidValue;
  return ps.mode == LP_BF16X3 ? dispatch_dma<LP_BF16X3>(ps, stream) : dispatch_dma<LP_BF16>(ps, stream);
}

hipError_t launch_to_lowp(const double* f, void* out, long plane_o, int split, const int dims[3], int ldo,
                          hipStream_t stream) {
  const long rows = (long)dims[0] * dims[1];
  if (rows <= 0) return hipSuccess;
  if (ldo < dims[2] || (split && plane_o < rows * ldo)) return hipErrorInvalidValue;
  if ((rows + 3) / 4 > 0x7fffffffL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((rows + 3) / 4)), block(256);
  if (split)
    dmak::to_lowp_kernel<2><<<grid, block, 0, stream>>>(f, (unsigned short*)out, plane_o, rows, dims[2], ldo);
  else
    dmak::to_lowp_kernel<1><<<grid, block, 0, stream>>>(f, (unsigned short*)out, plane_o, rows, dims[2], ldo);
  return hipGetLastError();
}

}  // namespace semfd
