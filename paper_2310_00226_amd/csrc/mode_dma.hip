// BF16 rotating mode products with direct global -> LDS loads.
//
// Same contraction as the FP32 passes (Y[l][a][b] = sum_k F[l][k] X[a][b][k],
// the axes rotating from pass to pass) for the two BF16 modes, organised for
// CDNA4:
//  * operand tiles move from HBM / L2 straight into LDS with
//    global_load_lds_dwordx4 (no VGPR staging), through a ring of STAGES
//    buffers; the loads of chunk c + STAGES - 1 are in flight while chunk c is
//    multiplied, and a wave waits (vmcnt) only for the chunk it is about to read;
//  * the ring stages are addressed with compile-time indices (the chunk loop is
//    unrolled by STAGES); the kernel orders DMA and LDS reads itself (vmcnt wait
//    + barrier per chunk), so the loads of later stages stay in flight;
//  * LDS rows are 64 bytes (32 BF16 = one 16x16x32 MFMA step) made of four
//    16-byte chunks placed at slot chunk ^ g(row), g(row) = ((row>>1)^(row>>2))&3,
//    which makes the fragment reads (16 rows x one chunk per 16 lanes)
//    bank-conflict-free for 32 and 64 four-byte banks;
//  * block tile 256 (l) x 256 (p), eight waves of 128 x 64;
//  * the output columns run over the padded output layout, p = a * ldy + b with
//    b < ldy, so that an output row (fixed l) of the tile is one contiguous
//    segment y[l * A * ldy + p]: the epilogue stages the tile in LDS and writes
//    it with 16-byte stores (padding columns b >= B receive finite values
//    computed from a repeated input row, which the next pass multiplies by zero
//    factor columns).
// Split BF16 (LP_BF16X3) keeps every operand as two BF16 planes (hi, lo) in
// HBM, so its intermediates load without conversion too.
//
// Contract of the operands (set up by the caller):
//  * tensor rows have a pitch ldx that is a multiple of 8 elements (16 bytes);
//    elements between K and ldx hold finite values (they meet zero factor
//    columns), and the second plane (split mode) starts xplane elements after
//    the first;
//  * the factor is [l][k] with pitch ldf (multiple of 8, >= 256-rounded L and
//    32-rounded K), 256-rounded L rows, zero outside L x K, second plane fplane
//    elements after the first;
//  * BF16 outputs have a pitch ldy that is a multiple of 8.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdint>

#include "kernels.h"

namespace semfd {

namespace dmak {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef unsigned u4_t __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;

constexpr int BM = 256, BN = 256, WL = 2, WP = 4;
constexpr int NTHREADS = 64 * WL * WP;  // 512
constexpr int TL = BM / WL, TP = BN / WP;  // 128 x 64 per wave
constexpr int FL = TL / 16, FP = TP / 16;  // 8 x 4 MFMA tiles
constexpr int BK = 32;                      // BF16 elements per chunk (64-byte LDS rows)
constexpr int ROWB = BK * 2;                // bytes per LDS row
constexpr int TILEB = BM * ROWB;            // bytes per operand tile (16 KB)
// epilogue staging: BF16 rows of 264 elements (16-byte aligned row starts) and
// FP32 rows of 260; in both, rows 4 apart start on different banks, so the
// MFMA output layout writes without conflicts
constexpr int EROW_H = 264, EROW_F = 260;
constexpr int EPIB = 256 * EROW_H * 2;  // 256 BF16 rows (>= 128 FP32 rows)
static_assert(128 * EROW_F * 4 <= EPIB, "FP32 staging fits");

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
  static constexpr int NS = MODE == LP_BF16X3 ? 2 : 1;
  static constexpr int STAGES = NS == 2 ? 2 : 4;
  static constexpr int STAGEB = NS * 2 * TILEB;  // factor + tensor tiles, all planes
  // DMA instructions per chunk per wave: each 1 KB instruction fills 16 rows
  static constexpr int DMA_PER_TILE = BM / 16 / (WL * WP);  // 2
  static constexpr int D = NS * 2 * DMA_PER_TILE;
  static constexpr int SMEM = STAGES * STAGEB > EPIB ? STAGES * STAGEB : EPIB;
};

template <int MODE, class TOut, int EPI>
__global__ __launch_bounds__(NTHREADS) void mode_rot_dma(const unsigned short* __restrict__ x, int ldx, long xplane,
                                                         long P, int K, TOut* __restrict__ y, int ldy, long yplane,
                                                         int A, int B, int L, const unsigned short* __restrict__ f,
                                                         int ldf, long fplane, long tiles_l, long ntiles,
                                                         long nblocks_padded, EpiLP epi) {
  typedef KCfg<MODE> C;
  constexpr int NS = C::NS, S = C::STAGES;
  __shared__ __attribute__((aligned(1024))) unsigned char smem[C::SMEM];
  unsigned char* const st0 = smem;
  unsigned char* const st1 = smem + C::STAGEB;
  unsigned char* const st2 = smem + (S > 2 ? 2 : 0) * C::STAGEB;
  unsigned char* const st3 = smem + (S > 3 ? 3 : 0) * C::STAGEB;

  const long t = xcd_tile(nblocks_padded);
  if (t >= ntiles) return;  // whole block leaves together, before any barrier
  const long lt = t % tiles_l;
  const long pt = t / tiles_l;
  const int l0 = (int)(lt * BM);
  const long p0 = pt * BN;
  const long Pp = (long)A * ldy;  // padded output columns

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = (wave / WP) * TL;
  const int wn = (wave % WP) * TP;
  const int nchunk = (K + BK - 1) / BK;

  // ---- DMA source addresses --------------------------------------------------
  // Instruction q (0, 1) of this wave fills tile rows 16*(2*wave + q) .. +15;
  // lane i writes LDS slot i % 4 of row 16*(2*wave + q) + i / 4 and therefore
  // fetches chunk (i % 4) ^ g(row) of that row.  Output column p = a * ldy + b
  // reads input row a * B + b; padding columns (b >= B) and columns past the end
  // read a valid row instead.
  const unsigned short* fsrc[2];
  const unsigned short* xsrc[2];
  int fchunk[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int row = 16 * (2 * wave + q) + lane / 4;
    fchunk[q] = ((lane & 3) ^ swz(row)) * 8;  // element offset of the chunk
    fsrc[q] = f + (size_t)(l0 + row) * ldf;
    const long pc = p0 + row;
    long pr = P - 1;
    if (pc < Pp) {
      const long a = pc / ldy;
      const long b = pc - a * ldy;
      pr = a * B + (b < B ? b : B - 1);
    }
    xsrc[q] = x + (size_t)pr * ldx;
  }
  auto issue = [&](unsigned char* stage, int c) {
    const int k0 = c * BK;
#pragma unroll
    for (int pl = 0; pl < NS; ++pl)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int ldsrow = 16 * (2 * wave + q);
        unsigned char* fdst = stage + pl * 2 * TILEB + ldsrow * ROWB;
        unsigned char* xdst = stage + pl * 2 * TILEB + TILEB + ldsrow * ROWB;
        // factor: padded, always in bounds; tensor: chunks past the row pitch
        // are redirected to the row start (finite data times zero factor columns)
        const int kf = k0 + fchunk[q];
        const int kx = kf < ldx ? kf : 0;
        __builtin_amdgcn_global_load_lds((const void*)(fsrc[q] + pl * fplane + kf), (lds_void*)fdst, 16, 0, 0);
        __builtin_amdgcn_global_load_lds((const void*)(xsrc[q] + pl * xplane + kx), (lds_void*)xdst, 16, 0, 0);
      }
  };

  f4_t acc[FL][FP];
#pragma unroll
  for (int i = 0; i < FL; ++i)
#pragma unroll
    for (int j = 0; j < FP; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

  const int fr = lane & 15, fg = lane >> 4;
  // fragment byte offsets within a tile (row-dependent swizzle)
  int aoff[FL], boff[FP];
#pragma unroll
  for (int i = 0; i < FL; ++i) {
    const int row = wm + 16 * i + fr;
    aoff[i] = row * ROWB + ((fg ^ swz(row)) << 4);
  }
#pragma unroll
  for (int j = 0; j < FP; ++j) {
    const int row = wn + 16 * j + fr;
    boff[j] = row * ROWB + ((fg ^ swz(row)) << 4);
  }
  auto compute = [&](const unsigned char* stage) {
    bf8_t a[FL], b[FP];
#pragma unroll
    for (int i = 0; i < FL; ++i) a[i] = *reinterpret_cast<const bf8_t*>(stage + aoff[i]);
#pragma unroll
    for (int j = 0; j < FP; ++j) b[j] = *reinterpret_cast<const bf8_t*>(stage + TILEB + boff[j]);
    if constexpr (NS == 2) {
      bf8_t alo[FL], blo[FP];
#pragma unroll
      for (int i = 0; i < FL; ++i) alo[i] = *reinterpret_cast<const bf8_t*>(stage + 2 * TILEB + aoff[i]);
#pragma unroll
      for (int j = 0; j < FP; ++j) blo[j] = *reinterpret_cast<const bf8_t*>(stage + 3 * TILEB + boff[j]);
      __builtin_amdgcn_sched_barrier(0);  // all fragment reads in flight before the first MFMA
      // products outermost: consecutive MFMAs write different accumulators
#pragma unroll
      for (int i = 0; i < FL; ++i)
#pragma unroll
        for (int j = 0; j < FP; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[i], b[j], acc[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < FL; ++i)
#pragma unroll
        for (int j = 0; j < FP; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], blo[j], acc[i][j], 0, 0, 0);
    } else {
      __builtin_amdgcn_sched_barrier(0);  // all fragment reads in flight before the first MFMA
    }
#pragma unroll
    for (int i = 0; i < FL; ++i)
#pragma unroll
      for (int j = 0; j < FP; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  };

  // ---- pipeline -----------------------------------------------------------------
  // Every step issues exactly D DMA instructions per wave (past the last chunk it
  // reloads the last chunk into the free stage, never read), so the number of
  // instructions in flight behind chunk c is always (S - 2) * D and one constant
  // vmcnt wait covers every step.
  const int clast = nchunk - 1;
  issue(st0, 0);
  if constexpr (S > 2) {
    issue(st1, 1 < clast ? 1 : clast);
    issue(st2, 2 < clast ? 2 : clast);
  }
  // One step: wait until this wave's DMAs of chunk c landed, barrier (every wave's
  // part landed, and every wave is done reading the stage about to be refilled),
  // refill that stage with chunk c + S - 1, multiply chunk c.
  auto step = [&](int c, unsigned char* cur, unsigned char* refill) {
    wait_vm<(S - 2) * C::D>();
    __builtin_amdgcn_s_barrier();
    issue(refill, c + S - 1 < clast ? c + S - 1 : clast);
    compute(cur);
  };
  for (int c = 0; c < nchunk; c += S) {
    if constexpr (S == 4) {
      step(c, st0, st3);
      if (c + 1 < nchunk) step(c + 1, st1, st0);
      if (c + 2 < nchunk) step(c + 2, st2, st1);
      if (c + 3 < nchunk) step(c + 3, st3, st2);
    } else {
      step(c, st0, st1);
      if (c + 1 < nchunk) step(c + 1, st1, st0);
    }
  }
  // drain the trailing reloads, then every wave is done with the ring
  wait_vm<0>();
  __syncthreads();

  // ---- epilogue: f32 16x16 layout: lane, reg r -> row 4*(lane/16) + r, col lane%16
  // The tile goes through LDS so that global stores are whole row segments.
  if constexpr (EPI == EPI_ACCUM) {
    // u += delta in FP64; two rounds of 128 rows staged as FP32
    float* sf = reinterpret_cast<float*>(smem);
    double dmax = 0.0, umax = 0.0;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      if (half) __syncthreads();  // the previous round's readers are done
      if (wm == half * TL) {
#pragma unroll
        for (int i = 0; i < FL; ++i)
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int j = 0; j < FP; ++j) sf[(16 * i + 4 * fg + r) * EROW_F + wn + 16 * j + fr] = acc[i][j][r];
      }
      __syncthreads();
      // batches of UB elements per thread: all their loads of u in flight at once
      constexpr int UB = 16;
      const int col = tid % BN;  // consecutive threads: consecutive columns
      const long pc = p0 + col;
#pragma unroll 1
      for (int it0 = 0; it0 < TL * BN / NTHREADS; it0 += UB) {
        double uo[UB];
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          const int row = (it0 + u) * (NTHREADS / BN) + tid / BN;
          const long l = l0 + half * TL + row;
          const bool in = l < L && pc < Pp;
          uo[u] = (in && !epi.first) ? (double)y[(size_t)l * Pp + pc] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          const int row = (it0 + u) * (NTHREADS / BN) + tid / BN;
          const long l = l0 + half * TL + row;
          if (l < L && pc < Pp) {
            const double dv = (double)sf[row * EROW_F + col];
            const double un = uo[u] + dv;
            y[(size_t)l * Pp + pc] = (TOut)un;
            // a NaN / Inf turns the norm into +Inf (fmax alone would drop NaN)
            dmax = fabs(dv) <= DBL_MAX ? fmax(dmax, fabs(dv)) : INFINITY;
            umax = fabs(un) <= DBL_MAX ? fmax(umax, fabs(un)) : INFINITY;
          }
        }
      }
    }
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
  } else {
    // BF16 planes (hi, then lo for split), optional spectral divide
    if constexpr (EPI == EPI_DIVIDE) {
      double dab[FP];
#pragma unroll
      for (int j = 0; j < FP; ++j) {
        const long pc = p0 + wn + 16 * j + fr;
        long a = 0, b = 0;
        if (pc < Pp) {
          a = pc / ldy;
          b = pc - a * ldy;
          if (b >= B) b = B - 1;  // padding column: any finite value
        }
        dab[j] = epi.l1[a] + epi.l2[b];
      }
#pragma unroll
      for (int i = 0; i < FL; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int l = l0 + wm + 16 * i + 4 * fg + r;
          const double dl = epi.l0[l < L ? l : L - 1];
#pragma unroll
          for (int j = 0; j < FP; ++j)
            acc[i][j][r] = __fdividef(acc[i][j][r], (float)spectral_den(dl + dab[j], epi.alpha, epi.b1, epi.b2));
        }
    }
    unsigned short* sh = reinterpret_cast<unsigned short*>(smem);
#pragma unroll
    for (int pl = 0; pl < NS; ++pl) {
      if (pl) __syncthreads();  // the previous round's readers are done
#pragma unroll
      for (int i = 0; i < FL; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int j = 0; j < FP; ++j) {
            const float w = acc[i][j][r];
            const __bf16 h = (__bf16)w;
            const __bf16 o = pl == 0 ? h : (__bf16)(w - (float)h);
            sh[(wm + 16 * i + 4 * fg + r) * EROW_H + wn + 16 * j + fr] = __builtin_bit_cast(unsigned short, o);
          }
      __syncthreads();
      TOut* __restrict__ yp = y + pl * yplane;
#pragma unroll 4
      for (int it = 0; it < BM * BN / 8 / NTHREADS; ++it) {
        const int idx = it * NTHREADS + tid;
        const int row = idx / (BN / 8), ch = idx % (BN / 8);
        const long l = l0 + row;
        const long pc = p0 + 8 * ch;
        if (l < L && pc < Pp)  // Pp is a multiple of 8: a chunk is wholly in or out
          *reinterpret_cast<u4_t*>(yp + (size_t)l * Pp + pc) =
              *reinterpret_cast<const u4_t*>(sh + row * EROW_H + 8 * ch);
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
  // must keep 16-byte chunks aligned, BF16 outputs 16-byte row segments
  const long pad256 = (ps.L + 255) / 256 * 256;
  const bool out_ok = ps.out_kind == 0 ? ps.ldy == ps.B : (ps.ldy % 8 == 0 && ps.ldy >= ps.B);
  return (ps.mode == LP_BF16 || ps.mode == LP_BF16X3) && ps.in_kind == 2 && ps.ldf >= pad256 &&
         ps.ldf % 8 == 0 && ps.ldx % 8 == 0 && ps.ldx >= ps.K && ps.ldf >= (ps.K + 31) / 32 * 32 && out_ok &&
         ps.P == (long)ps.A * ps.B;
}

template <int MODE, class TOut, int EPI>
static hipError_t launch_dma_t(const LpPass& ps, hipStream_t stream) {
  using namespace dmak;
  const long tiles_l = (ps.L + BM - 1) / BM;
  const long tiles_p = ((long)ps.A * ps.ldy + BN - 1) / BN;
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
