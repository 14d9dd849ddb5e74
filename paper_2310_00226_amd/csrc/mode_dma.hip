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
//    segment y[l * A * ldy + p] (padding columns b >= B receive finite values
//    computed from a repeated input row, which the next pass multiplies by zero
//    factor columns);
//  * the MFMAs take the tensor fragment as their first operand, so each lane
//    accumulates 4 consecutive output columns of one row: the epilogue stages the
//    tile in LDS with one 8-byte (BF16) or 16-byte (FP32) write per lane and block
//    and writes whole-row 16-byte segments.
// Split BF16 (LP_BF16X3) keeps every operand as two BF16 planes (hi, lo) in
// HBM, so its intermediates load without conversion too, and forms all four
// products hi*hi + hi*lo + lo*hi + lo*lo: the product of the two-term
// representations is then exact up to FP32 accumulation (dropping lo*lo, a
// systematic 2^-16 relative term, left the solve 1.3-1.8e-5 from FP64 and made
// the refinement of the n = 999 workload need a fourth iteration).
//
// Reflection-split ("folded") passes.  The 1D eigenvectors are symmetric or
// antisymmetric under the reflection of the axis, so a transform acts on the
// folded vector (v+_r = v_r + v_R(r), v-_r = v_r - v_R(r) over the orbit
// representatives r) as two half-size blocks.  A pass then has two contraction
// blocks: the l-tiles of block 1 contract the tensor's k in [0, K1) with factor
// rows from 0, those of block 2 contract k in [koff2, koff2 + K2) with factor rows
// from frow2; block 2's output rows follow block 1's L1 rows.  Output columns
// (the input row's second index b) are written in one of three layouts:
//  * COL_PLAIN: column b, padding columns from a repeated input row;
//  * COL_SPLIT: b is a folded mode index (b < bsym symmetric, else antisymmetric),
//    written at column b or bpad + (b - bsym) so that each block of the next
//    contraction starts on a 32-element boundary;
//  * COL_FOLD: b is a node index whose axis the next pass contracts: the tile's
//    columns are (representative, reflected node) pairs in adjacent lanes, and
//    the epilogue writes v+ at column r and v- at column bpad + r (a lane swap
//    gives each lane its partner's value).
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

#include <algorithm>
#include <cfloat>
#include <cstdint>

#include "kernels.h"

namespace semfd {

namespace dmak {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef unsigned u4_t __attribute__((ext_vector_type(4)));
typedef unsigned u2_t __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) void lds_void;

constexpr int BM = 256, BN = 256, WL = 2, WP = 4;
constexpr int NTHREADS = 64 * WL * WP;  // 512
constexpr int TL = BM / WL, TP = BN / WP;  // 128 x 64 per wave
constexpr int FL = TL / 16, FP = TP / 16;  // 8 x 4 MFMA tiles
constexpr int BK = 32;                      // BF16 elements per chunk (64-byte LDS rows)
constexpr int ROWB = BK * 2;                // bytes per LDS row
constexpr int TILEB = BM * ROWB;            // bytes per operand tile (16 KB)

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

// Kernel arguments of one pass (see LpPass).
struct DmaArgs {
  const unsigned short* x = nullptr;
  long xplane = 0, P = 0;
  int ldx = 0;
  void* y = nullptr;
  long yplane = 0;
  int ldy = 0;
  int A = 0, B = 0;
  const unsigned short* f = nullptr;
  long fplane = 0;
  int ldf = 0;
  int K1 = 0, K2 = 0, koff2 = 0, frow2 = 0, L1 = 0, L2 = 0;
  long tl1 = 0, tiles_l = 0, tiles_p = 0, ntiles = 0, nbp = 0;
  int group = 1;
  int persist = 0;
  int col = COL_PLAIN, bsym = 0, bpad = 0, bn = 0, bper = 0;
  EpiLP epi;
};

// Input b (second row index) of padded output column bo (COL_PLAIN, COL_SPLIT);
// padding columns take a valid neighbour.
__device__ __forceinline__ long in_col(long bo, const DmaArgs& g) {
  if (g.col == COL_SPLIT)
    return bo < g.bpad ? min(bo, (long)g.bsym - 1) : g.bsym + min(bo - g.bpad, (long)(g.B - g.bsym) - 1);
  return min(bo, (long)g.B - 1);
}

// epilogue staging: BF16 rows of 272 elements, FP32 rows of 264: row starts 8
// banks apart, so the 16 rows x 4 column groups of one 8-byte (16-byte) write
// instruction meet at most two to a bank
constexpr int EROW_H = 272, EROW_F = 264;
constexpr int EPIB = 256 * EROW_H * 2;  // 256 BF16 rows (>= 128 FP32 rows)
static_assert(128 * EROW_F * 4 <= EPIB, "FP32 staging fits");

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

// One 256 x 256 output tile t of a pass: DMA ring over the contraction, MFMAs,
// epilogue.  Every thread of the block calls it with the same t.
template <int MODE, class TOut, int EPI, int COL>
__device__ __forceinline__ void dma_tile(const DmaArgs& g, const long t, unsigned char* const smem) {
  typedef KCfg<MODE> C;
  constexpr int NS = C::NS, S = C::STAGES;
  unsigned char* const st0 = smem;
  unsigned char* const st1 = smem + C::STAGEB;
  unsigned char* const st2 = smem + (S > 2 ? 2 : 0) * C::STAGEB;
  unsigned char* const st3 = smem + (S > 3 ? 3 : 0) * C::STAGEB;
  // tile order: groups of `group` p-strips (the last one possibly shorter) step
  // through the l-tiles together, the strips of a group fastest
  const long per_group = g.tiles_l * g.group;
  const long grp = t / per_group;
  const long gsz = min((long)g.group, g.tiles_p - grp * g.group);
  const long rem = t - grp * per_group;
  const long lt = rem / gsz;
  const long pt = grp * g.group + (rem - lt * gsz);
  // contraction block of this l-tile: factor rows, tensor k range, output rows
  const bool blk2 = lt >= g.tl1;
  const long lb = blk2 ? lt - g.tl1 : lt;      // tile index inside the block
  const int frow0 = (blk2 ? g.frow2 : 0) + (int)(lb * BM);
  const int koff = blk2 ? g.koff2 : 0;
  const int K = blk2 ? g.K2 : g.K1;
  const int lrows = (int)min((long)BM, (long)(blk2 ? g.L2 : g.L1) - lb * BM);  // valid rows of the tile
  const int orow0 = (blk2 ? g.L1 : 0) + (int)(lb * BM);
  const long Pp = (long)g.A * g.ldy;  // padded output columns
  // COL_FOLD: tile pt = (a, block of 128 representatives); else 256 consecutive
  // padded output columns
  long fa = 0, fr0 = 0, p0 = 0;
  if constexpr (COL == COL_FOLD) {
    const long tpa = (g.bsym + 127) / 128;
    fa = pt / tpa;
    fr0 = (pt - fa * tpa) * 128;
  } else {
    p0 = pt * BN;
  }

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = (wave / WP) * TL;
  const int wn = (wave % WP) * TP;
  const int nchunk = (K + BK - 1) / BK;

  // ---- DMA source addresses --------------------------------------------------
  // Instruction q (0, 1) of this wave fills tile rows 16*(2*wave + q) .. +15;
  // lane i writes LDS slot i % 4 of row 16*(2*wave + q) + i / 4 and therefore
  // fetches chunk (i % 4) ^ g(row) of that row.  Output columns map to input rows
  // (a, b) as described above; padding columns and columns past the end read a
  // valid row instead.
  const unsigned short* fsrc[2];
  const unsigned short* xsrc[2];
  int fchunk[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int row = 16 * (2 * wave + q) + lane / 4;
    fchunk[q] = ((lane & 3) ^ swz(row)) * 8;  // element offset of the chunk
    fsrc[q] = g.f + (size_t)(frow0 + row) * g.ldf;
    long pr = g.P - 1;
    if constexpr (COL == COL_FOLD) {
      const int r = (int)min(fr0 + (row >> 1), (long)g.bsym - 1);
      const int b = (row & 1) ? (g.bper ? (g.bn - r) % g.bn : g.bn - 1 - r) : r;
      pr = fa * g.B + b;
    } else {
      const long pc = p0 + row;
      if (pc < Pp) {
        const long a = pc / g.ldy;
        const long bo = pc - a * g.ldy;
        pr = a * g.B + in_col(bo, g);
      }
    }
    xsrc[q] = g.x + (size_t)pr * g.ldx + koff;
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
        // are redirected to the block start (finite data times zero factor columns)
        const int kf = k0 + fchunk[q];
        const int kx = koff + kf < g.ldx ? kf : 0;
        __builtin_amdgcn_global_load_lds((const void*)(fsrc[q] + pl * g.fplane + kf), (lds_void*)fdst, 16, 0, 0);
        __builtin_amdgcn_global_load_lds((const void*)(xsrc[q] + pl * g.xplane + kx), (lds_void*)xdst, 16, 0, 0);
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
    if constexpr (NS == 2) {
      // split BF16: the tensor fragments (hi, lo) of all 4 column blocks stay in
      // registers; the factor fragments are read one 16-row block at a time, and the
      // block's 4 x 4 MFMAs (products lo*hi, hi*lo, lo*lo, hi*hi, each over the 4
      // column blocks, so that consecutive MFMAs write different accumulators)
      // cover the reads of the next block.  Holding all 24 fragments at once needs
      // more than the 256 registers a wave has at two waves per SIMD.  The tensor
      // fragment is the first operand, so that acc[i][j] holds D[p][l]: a lane
      // keeps 4 consecutive output columns p of one row l (see the epilogue).
      bf8_t bh[FP], bl[FP];
#pragma unroll
      for (int j = 0; j < FP; ++j) {
        bh[j] = *reinterpret_cast<const bf8_t*>(stage + TILEB + boff[j]);
        bl[j] = *reinterpret_cast<const bf8_t*>(stage + 3 * TILEB + boff[j]);
      }
#pragma unroll
      for (int i = 0; i < FL; ++i) {
        const bf8_t ah = *reinterpret_cast<const bf8_t*>(stage + aoff[i]);
        const bf8_t al = *reinterpret_cast<const bf8_t*>(stage + 2 * TILEB + aoff[i]);
#pragma unroll
        for (int j = 0; j < FP; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[j], al, acc[i][j], 0, 0, 0);
#pragma unroll
        for (int j = 0; j < FP; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl[j], ah, acc[i][j], 0, 0, 0);
#pragma unroll
        for (int j = 0; j < FP; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl[j], al, acc[i][j], 0, 0, 0);
#pragma unroll
        for (int j = 0; j < FP; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[j], ah, acc[i][j], 0, 0, 0);
      }
    } else {
      bf8_t a[FL], b[FP];
#pragma unroll
      for (int i = 0; i < FL; ++i) a[i] = *reinterpret_cast<const bf8_t*>(stage + aoff[i]);
#pragma unroll
      for (int j = 0; j < FP; ++j) b[j] = *reinterpret_cast<const bf8_t*>(stage + TILEB + boff[j]);
      __builtin_amdgcn_sched_barrier(0);  // all fragment reads in flight before the first MFMA
#pragma unroll
      for (int i = 0; i < FL; ++i)
#pragma unroll
        for (int j = 0; j < FP; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j], a[i], acc[i][j], 0, 0, 0);
    }
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
  // drain the trailing reloads (they target the free stage, never read)
  wait_vm<0>();

  // ---- epilogue ------------------------------------------------------------------
  // acc[i][j][r] = D[p][l] with l = wm + 16 i + (lane % 16) and p = wn + 16 j +
  // 4 (lane / 16) + r: every lane holds 4 consecutive output columns of one row.
  // The tile is staged in LDS (one 8-byte BF16 or 16-byte FP32 write per lane and
  // block) and leaves as 16-byte segments of whole output rows.
  const int pl0 = wn + 4 * fg;  // first of the lane's columns in each 16-column block
  __syncthreads();              // every wave is done with the ring
  if constexpr (sizeof(TOut) == 4) {
    // FP32 output, plain columns: two rounds of 128 rows
    float* sf = reinterpret_cast<float*>(smem);
    float* __restrict__ yp = reinterpret_cast<float*>(g.y);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      if (half) __syncthreads();  // the previous round's readers are done
      if (wm == half * TL) {
#pragma unroll
        for (int i = 0; i < FL; ++i)
#pragma unroll
          for (int j = 0; j < FP; ++j)
            *reinterpret_cast<f4_t*>(sf + (16 * i + fr) * EROW_F + pl0 + 16 * j) = acc[i][j];
      }
      __syncthreads();
#pragma unroll 4
      for (int it = 0; it < TL * BN / 4 / NTHREADS; ++it) {
        const int idx = it * NTHREADS + tid;
        const int row = idx / (BN / 4), ch = idx % (BN / 4);
        const int lr = half * TL + row;
        const long pc = p0 + 4 * ch;
        if (lr < lrows && pc < Pp)  // Pp is a multiple of 8: a chunk is wholly in or out
          *reinterpret_cast<f4_t*>(yp + (size_t)(orow0 + lr) * Pp + pc) =
              *reinterpret_cast<const f4_t*>(sf + row * EROW_F + 4 * ch);
      }
    }
  } else {
    if constexpr (EPI == EPI_DIVIDE) {
      // denominators alpha + b1 L + b2 L^2, L = lam_l + lam_a + lam_b, in FP32 (the
      // quotient is rounded to split BF16 anyway): one thread per tile column forms
      // lam_a + lam_b (in FP64, then rounded) and one per tile row fetches lam_l,
      // both into LDS behind the staging area
      float* const dcol = reinterpret_cast<float*>(smem + C::SMEM);
      float* const drow = dcol + BN;
      if (tid < BN) {
        const long c = p0 + tid;
        float v = 0.0f;
        if (c < Pp) {
          const long a = c / g.ldy;
          const long bo = c - a * g.ldy;
          v = (float)(g.epi.l1[a] + g.epi.l2[in_col(bo, g)]);
        }
        dcol[tid] = v;
      } else {
        const int lr = tid - BN;
        drow[lr] = (float)g.epi.l0[orow0 + (lr < lrows ? lr : lrows - 1)];
      }
      __syncthreads();
      const float al = (float)g.epi.alpha, b1 = (float)g.epi.b1, b2 = (float)g.epi.b2;
#pragma unroll
      for (int i = 0; i < FL; ++i) {
        const float dl = drow[wm + 16 * i + fr];
#pragma unroll
        for (int j = 0; j < FP; ++j) {
          const f4_t dab = *reinterpret_cast<const f4_t*>(dcol + pl0 + 16 * j);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            // hardware reciprocal (1 ulp): the quotient is rounded to BF16 next
            const float L = dl + dab[r];
            acc[i][j][r] *= __builtin_amdgcn_rcpf(al + L * (b1 + b2 * L));
          }
        }
      }
    }
    if constexpr (COL == COL_FOLD) {
      // columns 2q, 2q + 1 hold the representative and the reflected node of one
      // orbit: r = 0, 1 and r = 2, 3 become (v+, v-) of two consecutive orbits
#pragma unroll
      for (int i = 0; i < FL; ++i)
#pragma unroll
        for (int j = 0; j < FP; ++j) {
          const f4_t v = acc[i][j];
          acc[i][j] = f4_t{v[0] + v[1], v[2] + v[3], v[0] - v[1], v[2] - v[3]};
        }
    }
    unsigned short* sh = reinterpret_cast<unsigned short*>(smem);
    unsigned short* __restrict__ yh = reinterpret_cast<unsigned short*>(g.y);
#pragma unroll
    for (int pl = 0; pl < NS; ++pl) {
      if (pl) {
        __syncthreads();  // the previous round's readers are done
        // the lo round converts again instead of keeping the hi round's 128 BF16
        // values live next to the accumulators (which would spill)
#pragma unroll
        for (int i = 0; i < FL; ++i)
#pragma unroll
          for (int j = 0; j < FP; ++j) asm volatile("" : "+v"(acc[i][j]));
      }
#pragma unroll
      for (int i = 0; i < FL; ++i)
#pragma unroll
        for (int j = 0; j < FP; ++j) {
          unsigned w[2];
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            const float x0 = acc[i][j][2 * t], x1 = acc[i][j][2 * t + 1];
            const __bf16 h0 = (__bf16)x0, h1 = (__bf16)x1;
            const __bf16 o0 = pl == 0 ? h0 : (__bf16)(x0 - (float)h0);
            const __bf16 o1 = pl == 0 ? h1 : (__bf16)(x1 - (float)h1);
            w[t] = (unsigned)__builtin_bit_cast(unsigned short, o0) |
                   ((unsigned)__builtin_bit_cast(unsigned short, o1) << 16);
          }
          unsigned short* srow = sh + (16 * i + fr + wm) * EROW_H;
          if constexpr (COL == COL_FOLD) {
            // v+ of orbits c/2, c/2 + 1 to staging columns c/2.., v- to 128 + c/2..
            const int sc = (pl0 + 16 * j) >> 1;
            *reinterpret_cast<unsigned*>(srow + sc) = w[0];
            *reinterpret_cast<unsigned*>(srow + BN / 2 + sc) = w[1];
          } else {
            *reinterpret_cast<u2_t*>(srow + pl0 + 16 * j) = u2_t{w[0], w[1]};
          }
        }
      __syncthreads();
      unsigned short* __restrict__ yp = yh + pl * g.yplane;
#pragma unroll 4
      for (int it = 0; it < BM * BN / 8 / NTHREADS; ++it) {
        const int idx = it * NTHREADS + tid;
        const int row = idx / (BN / 8), ch = idx % (BN / 8);
        if (row >= lrows) continue;
        const size_t ybase = (size_t)(orow0 + row) * Pp;
        if constexpr (COL == COL_FOLD) {
          // chunk ch < 16: v+ columns fr0 + 8 ch; else v- columns bpad + fr0 + 8 (ch - 16)
          const long rc = fr0 + 8 * (ch & 15);
          if (rc < g.bpad)  // bpad is a multiple of 32: a chunk is wholly in or out
            *reinterpret_cast<u4_t*>(yp + ybase + fa * g.ldy + (ch >= 16 ? g.bpad : 0) + rc) =
                *reinterpret_cast<const u4_t*>(sh + row * EROW_H + 8 * ch);
        } else {
          const long pc = p0 + 8 * ch;
          if (pc < Pp)  // Pp is a multiple of 8: a chunk is wholly in or out
            *reinterpret_cast<u4_t*>(yp + ybase + pc) = *reinterpret_cast<const u4_t*>(sh + row * EROW_H + 8 * ch);
        }
      }
    }
  }
}

// A pass: one block per tile (persist = 0, blocks numbered XCD-aware), or one
// block per CU looping over tiles (persist = 1): each XCD takes a contiguous range
// of the tile numbering and its blocks stride through it, so that the stores of
// one tile drain while the next tile's first chunks stream in.
template <int MODE, class TOut, int EPI, int COL>
__global__ __launch_bounds__(NTHREADS) void mode_rot_dma(DmaArgs g) {
  typedef KCfg<MODE> C;
  // DIVIDE keeps the tile's 256 column and 256 row parts of the denominators
  // behind the staging area
  constexpr int SMEM_ALL = C::SMEM + (EPI == EPI_DIVIDE ? 2 * 256 * 4 : 0);
  __shared__ __attribute__((aligned(1024))) unsigned char smem[SMEM_ALL];
  if (!g.persist) {
    const long t = xcd_tile(g.nbp);
    if (t >= g.ntiles) return;  // whole block leaves together, before any barrier
    dma_tile<MODE, TOut, EPI, COL>(g, t, smem);
    return;
  }
  const long xcd = blockIdx.x & 7, j = blockIdx.x >> 3, nper = gridDim.x >> 3;
  const long per = (g.ntiles + 7) / 8;
  const long t_end = min((xcd + 1) * per, g.ntiles);
  for (long t = xcd * per + j; t < t_end; t += nper) {  // uniform over the block
    dma_tile<MODE, TOut, EPI, COL>(g, t, smem);
    __syncthreads();  // the next tile's DMAs overwrite the staging area
  }
}

// FP64 caller-layout array (rows of nz) -> BF16 hi (+ lo) planes with pitch ldo,
// padding zeroed; with fold, the rows are folded along z first (v+ at column r,
// v- at fpad + r, r < nrep; reflection n - 1 - r, or (n - r) mod n periodic),
// in FP64.  One wave per row.
template <int NS>
__global__ __launch_bounds__(256) void to_lowp_kernel(const double* __restrict__ f, unsigned short* __restrict__ o,
                                                      long plane_o, long rows, int nz, int ldo, int fold, int nrep,
                                                      int fpad, int per) {
  // a wave owns a row: FP64 values into LDS, folded in FP64, 16-byte BF16
  // stores; dynamic LDS of 4 nz doubles
  extern __shared__ double lowp_rows[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long row = (long)blockIdx.x * (blockDim.x >> 6) + wave;
  if (row >= rows) return;  // wave-uniform; no block-wide barrier below
  double* rv = lowp_rows + (size_t)wave * nz;
  const double* src = f + (size_t)row * nz;
  // 1024 values per round: all 16 loads of a lane in flight before the first
  // LDS store (a loop that stored each value as it arrived would wait on every load)
  for (int base = 0; base < nz; base += 1024) {
    double tv[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int e = base + 64 * t + lane;
      tv[t] = e < nz ? src[e] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int e = base + 64 * t + lane;
      if (e < nz) rv[e] = tv[t];
    }
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0);
  unsigned short* dst = o + (size_t)row * ldo;
  for (int c = lane; c < ldo / 8; c += 64) {
    u4_t hw, lw;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      unsigned hh = 0, ll = 0;
#pragma unroll
      for (int hlf = 0; hlf < 2; ++hlf) {
        const int e = 8 * c + 2 * t + hlf;
        double v = 0.0;
        if (!fold) {
          v = e < nz ? rv[e] : 0.0;
        } else {
          const bool minus = e >= fpad;
          const int r = minus ? e - fpad : e;
          if (r < nrep) {
            const int m = per ? (nz - r) % nz : nz - 1 - r;
            v = minus ? rv[r] - rv[m] : rv[r] + rv[m];
          }
        }
        const float fv = (float)v;
        const __bf16 h = (__bf16)fv;
        hh |= (unsigned)__builtin_bit_cast(unsigned short, h) << (16 * hlf);
        ll |= (unsigned)__builtin_bit_cast(unsigned short, (__bf16)(fv - (float)h)) << (16 * hlf);
      }
      hw[t] = hh;
      lw[t] = ll;
    }
    *reinterpret_cast<u4_t*>(dst + 8 * c) = hw;
    if (NS == 2) *reinterpret_cast<u4_t*>(dst + plane_o + 8 * c) = lw;
  }
}

__device__ __forceinline__ float bf_val(const unsigned short* p, long i, long plane, int ns) {
  float v = (float)__builtin_bit_cast(__bf16, p[i]);
  if (ns == 2) v += (float)__builtin_bit_cast(__bf16, p[i + plane]);
  return v;
}

// BF16 (split: hi + lo planes) rows of pitch ldi, nz values each -> the same rows
// folded along z (pitch ldo, v+ at r, v- at fpad + r), FP32 arithmetic.  A wave
// owns a row: the row's values come in as 16-byte loads into LDS (FP32, hi + lo
// combined), the folded values leave as 16-byte stores.  ldi and ldo are
// multiples of 8; dynamic LDS of 4 ldi floats (one row per wave).
template <int NS>
__global__ __launch_bounds__(256) void fold_lowp_kernel(const unsigned short* __restrict__ in, long plane_i, int ldi,
                                                        unsigned short* __restrict__ o, long plane_o, int ldo,
                                                        long rows, int nz, int nrep, int fpad, int per) {
  extern __shared__ float fold_rows[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long row = (long)blockIdx.x * 4 + wave;
  if (row >= rows) return;  // wave-uniform; no block-wide barrier below
  float* rv = fold_rows + (size_t)wave * ldi;
  const unsigned short* src = in + row * ldi;
  // 4 x 512 values per round, every load of a lane in flight before the LDS stores
  for (int base = 0; base < ldi / 8; base += 256) {
    u4_t hv[4], lv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = base + 64 * q + lane;
      hv[q] = lv[q] = u4_t{0u, 0u, 0u, 0u};
      if (c < ldi / 8) {
        hv[q] = *reinterpret_cast<const u4_t*>(src + 8 * c);
        if (NS == 2) lv[q] = *reinterpret_cast<const u4_t*>(src + plane_i + 8 * c);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = base + 64 * q + lane;
      if (c >= ldi / 8) continue;
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int hlf = 0; hlf < 2; ++hlf) {
          float v = __uint_as_float((hv[q][t] >> (16 * hlf)) << 16);
          if (NS == 2) v += __uint_as_float((lv[q][t] >> (16 * hlf)) << 16);
          rv[8 * c + 2 * t + hlf] = v;
        }
    }
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0);
  unsigned short* dst = o + (size_t)row * ldo;
  for (int c = lane; c < ldo / 8; c += 64) {
    u4_t hw, lw;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      unsigned hh = 0, ll = 0;
#pragma unroll
      for (int hlf = 0; hlf < 2; ++hlf) {
        const int e = 8 * c + 2 * t + hlf;
        const bool minus = e >= fpad;
        const int r = minus ? e - fpad : e;
        float v = 0.0f;
        if (r < nrep) {
          const int m = per ? (nz - r) % nz : nz - 1 - r;
          v = minus ? rv[r] - rv[m] : rv[r] + rv[m];
        }
        const __bf16 h = (__bf16)v;
        hh |= (unsigned)__builtin_bit_cast(unsigned short, h) << (16 * hlf);
        ll |= (unsigned)__builtin_bit_cast(unsigned short, (__bf16)(v - (float)h)) << (16 * hlf);
      }
      hw[t] = hh;
      lw[t] = ll;
    }
    *reinterpret_cast<u4_t*>(dst + 8 * c) = hw;
    if (NS == 2) *reinterpret_cast<u4_t*>(dst + plane_o + 8 * c) = lw;
  }
}

// u (+)= the unfolded correction.  d holds the correction with every axis in the
// folded node form: index e_r (r < nrep) then o_r (nrep + r) per axis, FP32, rows
// (x'', y'') of pitch ldd (z'' contiguous).  Node i of an axis takes e_r + s o_r
// with r its orbit representative and s = +1 (i = r) or -1 (i = R(r)).  A thread
// owns one orbit {x, R(x)} x {y, R(y)} x {z, R(z)}: it reads the 8 values of the
// orbit once and writes its (up to 8) nodes.  first = 1: u = correction.  norms
// (may be null): atomic max of |delta| and |u| as FP64 bit patterns.
struct UnfoldAxis {
  int n, nrep, per;
};
__device__ __forceinline__ int refl_node(int r, const UnfoldAxis& a) { return a.per ? (a.n - r) % a.n : a.n - 1 - r; }

// NT threads per block (128, 256 or 512): the launch takes the smallest that
// covers a row's nrep_z representatives in one pass (or 512)
template <int NT, bool DOT>
__global__ __launch_bounds__(NT) void unfold_accum_kernel(const float* __restrict__ d, int ldd, double* __restrict__ u,
                                                           UnfoldAxis ax, UnfoldAxis ay, UnfoldAxis az, int first,
                                                           unsigned long long* __restrict__ norms, UnfoldDot dot) {
  // blocks stride over the orbit rows (x_r, y_r), threads over z_r; one atomic
  // pair per block for the norms
  constexpr int NW = NT / 64;
  __shared__ double red[2][NW];
  double dmax = 0.0, umax = 0.0;
  double s0 = 0.0, s1 = 0.0;  // DOT: <r, u>_M and <u, q>_M of this thread's nodes
  const long rows = (long)ax.nrep * ay.nrep;
  const int ny2 = 2 * ay.nrep;
  for (long row = blockIdx.x; row < rows; row += gridDim.x) {
    const int xr = (int)(row / ay.nrep), yr = (int)(row - (long)xr * ay.nrep);
    const int xs[2] = {xr, refl_node(xr, ax)}, ys[2] = {yr, refl_node(yr, ay)};
    for (int zr = threadIdx.x; zr < az.nrep; zr += NT) {
      float v[2][2][2];
#pragma unroll
      for (int ex = 0; ex < 2; ++ex)
#pragma unroll
        for (int ey = 0; ey < 2; ++ey)
#pragma unroll
          for (int ez = 0; ez < 2; ++ez)
            v[ex][ey][ez] = d[((size_t)(xr + ex * ax.nrep) * ny2 + (yr + ey * ay.nrep)) * ldd + zr + ez * az.nrep];
      const int zs[2] = {zr, refl_node(zr, az)};
#pragma unroll
      for (int sx = 0; sx < 2; ++sx) {
        if (sx && xs[1] == xs[0]) continue;
#pragma unroll
        for (int sy = 0; sy < 2; ++sy) {
          if (sy && ys[1] == ys[0]) continue;
#pragma unroll
          for (int sz = 0; sz < 2; ++sz) {
            if (sz && zs[1] == zs[0]) continue;
            double dv = 0.0;
#pragma unroll
            for (int ex = 0; ex < 2; ++ex)
#pragma unroll
              for (int ey = 0; ey < 2; ++ey)
#pragma unroll
                for (int ez = 0; ez < 2; ++ez) {
                  const int neg = (ex & sx) ^ (ey & sy) ^ (ez & sz);
                  dv += neg ? -(double)v[ex][ey][ez] : (double)v[ex][ey][ez];
                }
            const size_t gi = ((size_t)xs[sx] * ay.n + ys[sy]) * az.n + zs[sz];
            const double un = (first ? 0.0 : u[gi]) + dv;
            u[gi] = un;
            if constexpr (DOT) {
              const double m = dot.mx[xs[sx]] * dot.my[ys[sy]] * dot.mz[zs[sz]];
              s0 += m * dot.r[gi] * un;
              s1 += m * un * dot.q[gi];
            }
            // a NaN / Inf turns the norm into +Inf (fmax alone would drop NaN)
            dmax = fabs(dv) <= DBL_MAX ? fmax(dmax, fabs(dv)) : INFINITY;
            umax = fabs(un) <= DBL_MAX ? fmax(umax, fabs(un)) : INFINITY;
          }
        }
      }
    }
  }
  if constexpr (DOT) {  // fixed-order block sums (waves, then the NW wave sums)
#pragma unroll
    for (int s2 = 32; s2 >= 1; s2 >>= 1) {
      s0 += __shfl_xor(s0, s2);
      s1 += __shfl_xor(s1, s2);
    }
    __shared__ double dsum[2][NW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
      dsum[0][wave] = s0;
      dsum[1][wave] = s1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double t0 = 0.0, t1 = 0.0;
      for (int w2 = 0; w2 < NW; ++w2) {
        t0 += dsum[0][w2];
        t1 += dsum[1][w2];
      }
      dot.partial[2 * (size_t)blockIdx.x] = t0;
      dot.partial[2 * (size_t)blockIdx.x + 1] = t1;
    }
  }
  if (norms) {
#pragma unroll
    for (int s2 = 32; s2 >= 1; s2 >>= 1) {
      dmax = fmax(dmax, __shfl_xor(dmax, s2));
      umax = fmax(umax, __shfl_xor(umax, s2));
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
      red[0][wave] = dmax;
      red[1][wave] = umax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < NW; ++w) {
        dmax = fmax(dmax, red[0][w]);
        umax = fmax(umax, red[1][w]);
      }
      atomicMax(norms, (unsigned long long)__double_as_longlong(dmax));
      atomicMax(norms + 1, (unsigned long long)__double_as_longlong(umax));
    }
  }
}

}  // namespace dmak

bool dma_supported(const LpPass& ps) {
  // whole 256-row factor tiles must exist in the padded factor; the tensor pitch
  // keeps 16-byte chunks aligned, outputs 16-byte row segments; every block
  // contracts at least one element inside the row pitch
  const bool two = ps.K2 > 0;
  const long rows1 = (ps.L + 255) / 256 * 256;
  if (!(ps.mode == LP_BF16 || ps.mode == LP_BF16X3) || ps.in_kind != 2) return false;
  if (ps.ldf % 8 || ps.ldx % 8 || ps.ldy % 8 || ps.ldy < 1 || ps.K < 1 || ps.L < 1) return false;
  if (ps.ldx < (ps.K + 31) / 32 * 32 || ps.ldf < (ps.K + 31) / 32 * 32) return false;
  if (two && (ps.koff2 % 8 || ps.koff2 + (ps.K2 + 31) / 32 * 32 > ps.ldx || ps.ldf < (ps.K2 + 31) / 32 * 32 ||
              ps.frow2 < rows1 || ps.L2 < 1))
    return false;
  if (!(ps.out_kind == 2 || (ps.out_kind == 1 && ps.epi_kind == EPI_STORE && ps.col == COL_PLAIN))) return false;
  if (ps.P != (long)ps.A * ps.B || ps.A < 1 || ps.B < 1) return false;
  if (ps.col == COL_PLAIN) return ps.ldy >= ps.B;
  if (ps.col == COL_SPLIT) return ps.bsym >= 1 && ps.bsym <= ps.B && ps.bpad % 32 == 0 && ps.bpad >= ps.bsym &&
                                  ps.ldy >= ps.bpad + (ps.B - ps.bsym + 31) / 32 * 32 && ps.ldy >= ps.bpad + 32;
  if (ps.col == COL_FOLD) return ps.epi_kind == EPI_STORE && ps.bn == ps.B && ps.bsym >= 1 && ps.bsym <= ps.B &&
                                 ps.bpad % 32 == 0 && ps.bpad >= ps.bsym && ps.ldy >= 2 * ps.bpad;
  return false;
}

template <int MODE, class TOut, int EPI, int COL>
static hipError_t launch_dma_t(const LpPass& ps, hipStream_t stream) {
  using namespace dmak;
  DmaArgs g;
  g.x = (const unsigned short*)ps.x;
  g.xplane = ps.xplane;
  g.P = ps.P;
  g.ldx = ps.ldx;
  g.y = ps.y;
  g.yplane = ps.yplane;
  g.ldy = ps.ldy;
  g.A = ps.A;
  g.B = ps.B;
  g.f = (const unsigned short*)ps.f_hi;
  g.fplane = ps.fplane;
  g.ldf = ps.ldf;
  g.K1 = ps.K;
  g.L1 = ps.L;
  g.K2 = ps.K2;
  g.koff2 = ps.koff2;
  g.frow2 = ps.frow2;
  g.L2 = ps.L2;
  g.col = ps.col;
  g.bsym = ps.bsym;
  g.bpad = ps.bpad;
  g.bn = ps.bn;
  g.bper = ps.bper;
  g.epi = ps.epi;
  g.tl1 = (ps.L + BM - 1) / BM;
  g.tiles_l = g.tl1 + (ps.K2 > 0 ? (ps.L2 + BM - 1) / BM : 0);
  const long tiles_p =
      COL == COL_FOLD ? (long)ps.A * ((ps.bsym + 127) / 128) : ((long)ps.A * ps.ldy + BN - 1) / BN;
  g.tiles_p = tiles_p;
  g.ntiles = g.tiles_l * tiles_p;
  // tile_group: g in {1, 2, 4} (one block per tile) or DMA_PERSIST + g (one block
  // per CU looping over the tiles)
  const int tg = ps.tile_group >= 1 ? ps.tile_group : 1;
  g.persist = tg > DMA_PERSIST ? 1 : 0;
  g.group = g.persist ? tg - DMA_PERSIST : tg;
  g.nbp = ((g.ntiles + 7) / 8) * 8;
  if (g.ntiles == 0) return hipSuccess;
  if (g.nbp > 0x7fffffffL) return hipErrorInvalidValue;
  long grid = g.nbp;
  if (g.persist) {
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const long full = (long)(cus > 8 ? cus : 8) / 8 * 8;  // one block per CU, every XCD alike
    grid = full < g.nbp ? full : g.nbp;
  }
  mode_rot_dma<MODE, TOut, EPI, COL><<<dim3((unsigned)grid), dim3(NTHREADS), 0, stream>>>(g);
  return hipGetLastError();
}

template <int MODE>
static hipError_t dispatch_dma(const LpPass& ps, hipStream_t s) {
  if (ps.out_kind == 1) return launch_dma_t<MODE, float, EPI_STORE, COL_PLAIN>(ps, s);
  if (ps.epi_kind == EPI_DIVIDE) {
    if (ps.col == COL_SPLIT) return launch_dma_t<MODE, unsigned short, EPI_DIVIDE, COL_SPLIT>(ps, s);
    return launch_dma_t<MODE, unsigned short, EPI_DIVIDE, COL_PLAIN>(ps, s);
  }
  if (ps.epi_kind != EPI_STORE) return hipErrorInvalidValue;
  if (ps.col == COL_FOLD) return launch_dma_t<MODE, unsigned short, EPI_STORE, COL_FOLD>(ps, s);
  if (ps.col == COL_SPLIT) return launch_dma_t<MODE, unsigned short, EPI_STORE, COL_SPLIT>(ps, s);
  return launch_dma_t<MODE, unsigned short, EPI_STORE, COL_PLAIN>(ps, s);
}

hipError_t launch_mode_dma(const LpPass& ps, hipStream_t stream) {
  if (!dma_supported(ps)) return hipErrorInvalidValue;
  return ps.mode == LP_BF16X3 ? dispatch_dma<LP_BF16X3>(ps, stream) : dispatch_dma<LP_BF16>(ps, stream);
}

hipError_t launch_to_lowp(const double* f, void* out, long plane_o, int split, const int dims[3], int ldo,
                          const FoldAxis* fold, hipStream_t stream) {
  const long rows = (long)dims[0] * dims[1];
  if (rows <= 0) return hipSuccess;
  const int need = fold ? 2 * fold->pad : dims[2];
  if (ldo < need || ldo % 8 || dims[2] > 8192 || (split && plane_o < rows * ldo)) return hipErrorInvalidValue;
  if (rows == 0) return hipSuccess;
  // rows per block: at most 64 KB of LDS
  const int rpb = dims[2] <= 2048 ? 4 : dims[2] <= 4096 ? 2 : 1;
  if ((rows + rpb - 1) / rpb > 0x7fffffffL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((rows + rpb - 1) / rpb)), block(64 * rpb);
  const size_t lds = rpb * sizeof(double) * (size_t)dims[2];
  const int fo = fold ? 1 : 0, nr = fold ? fold->nrep : 0, fp = fold ? fold->pad : 0, pr = fold ? fold->per : 0;
  if (split)
    dmak::to_lowp_kernel<2><<<grid, block, lds, stream>>>(f, (unsigned short*)out, plane_o, rows, dims[2], ldo, fo, nr,
                                                        fp, pr);
  else
    dmak::to_lowp_kernel<1><<<grid, block, lds, stream>>>(f, (unsigned short*)out, plane_o, rows, dims[2], ldo, fo, nr,
                                                        fp, pr);
  return hipGetLastError();
}

hipError_t launch_fold_lowp(const void* in, long plane_i, int ldi, void* out, long plane_o, int ldo, int split,
                            const int dims[3], const FoldAxis& fold, hipStream_t stream) {
  const long rows = (long)dims[0] * dims[1];
  if (rows <= 0) return hipSuccess;
  if (ldi < dims[2] || ldo < 2 * fold.pad || fold.pad < fold.nrep || ldi % 8 || ldo % 8 || ldi > 8192 ||
      (split && (plane_o < rows * ldo || plane_i < rows * ldi)))
    return hipErrorInvalidValue;
  if ((rows + 3) / 4 > 0x7fffffffL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((rows + 3) / 4)), block(256);
  const size_t lds = 4 * sizeof(float) * (size_t)ldi;
  if (split)
    dmak::fold_lowp_kernel<2><<<grid, block, lds, stream>>>((const unsigned short*)in, plane_i, ldi,
                                                          (unsigned short*)out, plane_o, ldo, rows, dims[2],
                                                          fold.nrep, fold.pad, fold.per);
  else
    dmak::fold_lowp_kernel<1><<<grid, block, lds, stream>>>((const unsigned short*)in, plane_i, ldi,
                                                          (unsigned short*)out, plane_o, ldo, rows, dims[2],
                                                          fold.nrep, fold.pad, fold.per);
  return hipGetLastError();
}

template <int NT>
static hipError_t unfold_launch(const float* d, int ldd, double* u, const dmak::UnfoldAxis& ax,
                                const dmak::UnfoldAxis& ay, const dmak::UnfoldAxis& az, int first,
                                unsigned long long* norms, hipStream_t stream, const UnfoldDot* dot, long rows) {
  if (dot) {
    dmak::unfold_accum_kernel<NT, true><<<dim3((unsigned)dot->blocks), dim3(NT), 0, stream>>>(d, ldd, u, ax, ay, az,
                                                                                           first, norms, *dot);
    return hipGetLastError();
  }
  const unsigned grid = (unsigned)std::min<long>(rows, 8192);
  if (grid == 0) return hipSuccess;
  dmak::unfold_accum_kernel<NT, false><<<dim3(grid), dim3(NT), 0, stream>>>(d, ldd, u, ax, ay, az, first, norms,
                                                                            UnfoldDot());
  return hipGetLastError();
}

hipError_t launch_unfold_accum(const float* d, int ldd, double* u, const int dims[3], const FoldAxis fold[3],
                               int first, unsigned long long* norms, hipStream_t stream, const UnfoldDot* dot) {
  if (ldd < 2 * fold[2].nrep) return hipErrorInvalidValue;
  const dmak::UnfoldAxis ax{dims[0], fold[0].nrep, fold[0].per}, ay{dims[1], fold[1].nrep, fold[1].per},
      az{dims[2], fold[2].nrep, fold[2].per};
  const long rows = (long)fold[0].nrep * fold[1].nrep;
  if (dot && (!first || !dot->r || !dot->q || !dot->mx || !dot->my || !dot->mz || !dot->partial || dot->blocks < 1 ||
              dot->blocks != std::min<long>(rows, dot->blocks)))
    return hipErrorInvalidValue;
  if (az.nrep > 256) return unfold_launch<512>(d, ldd, u, ax, ay, az, first, norms, stream, dot, rows);
  if (az.nrep > 128) return unfold_launch<256>(d, ldd, u, ax, ay, az, first, norms, stream, dot, rows);
  return unfold_launch<128>(d, ldd, u, ax, ay, az, first, norms, stream, dot, rows);
}

}  // namespace semfd
