// FP64 mode-product kernels on CDNA4 matrix cores (v_mfma_f64_16x16x4f64).
//
// A "mode product" contracts one axis of a 3D nodal array with an n x n factor
// (paper Sec. 2.4, eq. tensorprod and the three-statement listing; eq.
// 3D-Poisson applies three of them forward and three backward).  Viewing the
// row-major tensor as X[p][m][q] (p = outer axes, m = contracted axis of length
// L, q = inner axes), every pass computes
//        Y[p][l][q] = sum_m A[l][m] X[p][m][q].
// The factor is stored by the plan as G[m][l] = A[l][m], zero-padded to a
// multiple of 128 in both dimensions, so tile loads of G need no bounds checks
// and padded contraction indices contribute exactly zero.
//
// Two tile shapes:
//   NN (q extent > 1: the x and y axes)  C = G^T-tile x X_p-tile
//        GEMM rows = l (M = L), cols = q (N = Q), batch = p.
//   NT (q extent = 1: the contiguous z axis)  C = X-tile x G-tile
//        GEMM rows = p (M = P), cols = l (N = L).
//
// Block = 256 threads = 4 waves in a 2 x 2 arrangement; block tile 128 x 128,
// each wave 64 x 64 = 4 x 4 MFMA tiles of 16 x 16.  Contraction chunks of 16 are
// staged through double-buffered LDS.  Epilogues: plain store, the eigenvalue
// divide of eq. 3D-Poisson (fused into the x-axis forward pass), or accumulate
// into FP64 (solution update of iterative refinement).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace semfd {

typedef double d4_t __attribute__((ext_vector_type(4)));

namespace f64k {

constexpr int BM = 128, BN = 128, BK = 16;
constexpr int NT_THREADS = 256;
constexpr int LDG = BN + 16;    // [BK][LDG] tiles: rows offset by 16 doubles mod 32 -> no bank clash
constexpr int LDT = BK + 2;     // [BM][LDT] tensor tile of the NT shape
constexpr int TILE_G = BK * LDG;
constexpr int TILE_T_NT = BM * LDT;

// XCD-aware tile numbering: hardware hands consecutive block ids to the 8 XCDs
// in turn; give each XCD a contiguous run of tiles so that the tiles sharing one
// tensor strip (which differ only in the fastest tile index) run together and
// hit the same L2.
__device__ __forceinline__ long xcd_tile(long nblocks_padded) {
  const long per = nblocks_padded / 8;
  return (long)(blockIdx.x % 8) * per + (long)(blockIdx.x / 8);
}

// ---------------------------------------------------------------------------
// NN: Y[p][l][q] = sum_m G[m][l] X[p][m][q]
// ---------------------------------------------------------------------------
template <int EPI>
__global__ __launch_bounds__(NT_THREADS, 2) void mode_nn_f64(const double* __restrict__ x, double* __restrict__ y,
                                                             const double* __restrict__ g, int ldg, long P, int K,
                                                             int L, int ldxa, int ldya, long Q, long tiles_l,
                                                             long tiles_q, long ntiles, long nblocks_padded,
                                                             EpiArgs epi) {
  __shared__ double lds[2 * (TILE_G + TILE_G)];
  const long t = xcd_tile(nblocks_padded);
  if (t >= ntiles) return;
  const long lt = t % tiles_l;
  const long rest = t / tiles_l;
  const long qt = rest % tiles_q;
  const long p = rest / tiles_q;
  const int l0 = (int)(lt * BM);
  const long q0 = qt * BN;
  const double* __restrict__ xp = x + (size_t)p * ldxa * Q;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * 64;  // wave row offset within the tile (l)
  const int wn = (wave & 1) * 64;   // wave col offset within the tile (q)

  // global -> register staging: element e = 0..7 of this thread covers row
  // kk = tid/64 + 4*(e>>1), col c = tid%64 + 64*(e&1) of a [BK][128] tile.  Loads
  // are branch-free: tensor columns past Q are clamped to a valid address (they
  // only feed output columns that are never stored); contraction rows past K are
  // clamped and zeroed (the padded factor rows are zero too).
  // The rows of each wave are wave-uniform (row pointers in scalar registers,
  // 32-bit lane offsets).
  double rg[8], rx[8];
  const int nchunk = (K + BK - 1) / BK;
  const int r0 = __builtin_amdgcn_readfirstlane(tid >> 6), c0 = tid & 63;
  const unsigned qa = (unsigned)(q0 + c0 < Q ? q0 + c0 : Q - 1);
  const unsigned qb = (unsigned)(q0 + c0 + 64 < Q ? q0 + c0 + 64 : Q - 1);
  const double* __restrict__ gw = g + (size_t)r0 * ldg + l0;

  auto load_chunk = [&](int c) {
    const int m0 = c * BK;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double* __restrict__ gr = gw + (size_t)(m0 + 4 * j) * ldg;
      rg[2 * j] = gr[c0];
      rg[2 * j + 1] = gr[c0 + 64];
      const int m = m0 + r0 + 4 * j;
      const int mc = m < K ? m : K - 1;
      const double* __restrict__ xr = xp + (size_t)mc * Q;  // (K >= 1 when loading)
      if (epi.fold) {  // uniform: v+ or v- of the unfolded axis at representative mc + roff
        const int rr = mc + epi.roff;
        xr = xp + (size_t)rr * Q;
        const double* __restrict__ xm = xp + (size_t)reflect_node(rr, epi.rn, epi.rper) * Q;
        const double a0 = xr[qa], a1 = xr[qb], b0 = xm[qa], b1 = xm[qb];
        rx[2 * j] = epi.fold == 1 ? a0 + b0 : a0 - b0;
        rx[2 * j + 1] = epi.fold == 1 ? a1 + b1 : a1 - b1;
      } else {
        rx[2 * j] = xr[qa];
        rx[2 * j + 1] = xr[qb];
      }
    }
  };
  // the zeroing of rows past K happens here, after the MFMA block, so that no wait
  // for the loads in flight is needed before it
  auto store_chunk = [&](int buf, int c) {
    double* sa = lds + buf * (2 * TILE_G);
    double* sb = sa + TILE_G;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kk = r0 + 4 * j;
      const bool ok = c * BK + kk < K;
      sa[kk * LDG + c0] = rg[2 * j];
      sa[kk * LDG + c0 + 64] = rg[2 * j + 1];
      sb[kk * LDG + c0] = ok ? rx[2 * j] : 0.0;
      sb[kk * LDG + c0 + 64] = ok ? rx[2 * j + 1] : 0.0;
    }
  };

  d4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

  const int fr = lane & 15, fk = lane >> 4;
  auto compute_chunk = [&](int buf) {
    const double* sa = lds + buf * (2 * TILE_G);
    const double* sb = sa + TILE_G;
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = sa[(ks * 4 + fk) * LDG + wm + 16 * i + fr];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = sb[(ks * 4 + fk) * LDG + wn + 16 * j + fr];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  };

  // steady state: loads of chunk c+1 are in flight while chunk c is multiplied
  // (K = 0, an empty antisymmetric block, leaves the accumulators at zero)
  if (nchunk > 0) {
    load_chunk(0);
    store_chunk(0, 0);
    __syncthreads();
    for (int c = 0; c + 1 < nchunk; ++c) {
      load_chunk(c + 1);
      // keep the LDS stores (which wait for the loads) after the whole MFMA block
      __builtin_amdgcn_sched_barrier(0);
      compute_chunk(c & 1);
      __builtin_amdgcn_sched_barrier(0);
      store_chunk((c + 1) & 1, c + 1);
      __syncthreads();
    }
    compute_chunk((nchunk - 1) & 1);
  }

  // f64 16x16 accumulator layout: lane, register r  ->  row 4r + lane/16, col lane%16
  double* __restrict__ yp = y + (size_t)p * ldya * Q;
  double cden[4] = {0.0, 0.0, 0.0, 0.0};
  if constexpr (EPI == EPI_DIVIDE || EPI == EPI_SPECTRAL) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long q = q0 + wn + 16 * j + fr;
      const int qi = (int)(q < Q ? q : Q - 1);
      const int jy = qi / (int)epi.nz;
      cden[j] = epi.ly[jy] + epi.lz[qi - jy * (int)epi.nz];  // partial eigenvalue sum
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int l = l0 + wm + 16 * i + 4 * r + fk;
      if (l >= L) continue;
      // EPI_UNFOLD: row l holds o of representative lr = l + roff, whose reflected
      // row takes e - o
      const int lr = EPI == EPI_UNFOLD ? l + epi.roff : l;
      const int lm = EPI == EPI_UNFOLD ? reflect_node(lr, epi.rn, epi.rper) : l;
      double* __restrict__ yrow = yp + (size_t)lr * Q;
      double* __restrict__ ymrow = yp + (size_t)lm * Q;
      const double lxl = (EPI == EPI_DIVIDE || EPI == EPI_SPECTRAL) ? epi.lx[l] : 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const long q = q0 + wn + 16 * j + fr;
        if (q >= Q) continue;
        const double v = acc[i][j][r];
        if constexpr (EPI == EPI_STORE) yrow[q] = v;
        else if constexpr (EPI == EPI_DIVIDE) yrow[q] = v / spectral_den(lxl + cden[j], epi.alpha, epi.b1, epi.b2);
        else if constexpr (EPI == EPI_SPECTRAL) yrow[q] = spectral_mul(v, lxl + cden[j], epi);
        else if constexpr (EPI == EPI_UNFOLD) {
          const double e = yrow[q];
          yrow[q] = e + v;
          if (lm != lr) ymrow[q] = e - v;
        } else yrow[q] += v;
      }
    }
}

// ---------------------------------------------------------------------------
// NT: Y[p][l] = sum_m X[p][m] G[m][l]
// ---------------------------------------------------------------------------
template <int EPI>
__global__ __launch_bounds__(NT_THREADS, 2) void mode_nt_f64(const double* __restrict__ x, double* __restrict__ y,
                                                             const double* __restrict__ g, int ldg, long P, int K,
                                                             int L, int ldxa, int ldya, long tiles_l, long ntiles,
                                                             long nblocks_padded, EpiArgs epi) {
  __shared__ double lds[2 * (TILE_T_NT + TILE_G)];
  const long t = xcd_tile(nblocks_padded);
  if (t >= ntiles) return;
  const long lt = t % tiles_l;
  const long pt = t / tiles_l;
  const int l0 = (int)(lt * BN);
  const long p0 = pt * BM;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * 64;  // rows: p
  const int wn = (wave & 1) * 64;   // cols: l

  // Factor tile [BK][128] as in the NN shape; tensor tile [128][BK]: element e of
  // this thread is row r = tid/16 + 16 e, contraction column tid%16.  Rows past P
  // are clamped to a valid address (their outputs are never stored); contraction
  // columns past K are clamped and zeroed.
  // Uniform tile base, 32-bit lane offsets (128 rows x ldxa < 2^32 elements).
  double rg[8], rx[8];
  const int nchunk = (K + BK - 1) / BK;
  const int r0 = __builtin_amdgcn_readfirstlane(tid >> 6), c0 = tid & 63;
  const double* __restrict__ gw = g + (size_t)r0 * ldg + l0;
  const int tr = tid >> 4, tc = tid & 15;
  const double* __restrict__ tb = x + (size_t)p0 * ldxa;
  const int rmax = (int)(P - 1 - p0);
  unsigned xoff[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int rr = tr + 16 * e;
    xoff[e] = (unsigned)(rr < rmax ? rr : rmax) * (unsigned)ldxa;
  }
  auto load_chunk = [&](int c) {
    const int m0 = c * BK;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double* __restrict__ gr = gw + (size_t)(m0 + 4 * j) * ldg;
      rg[2 * j] = gr[c0];
      rg[2 * j + 1] = gr[c0 + 64];
    }
    const int m = m0 + tc;
    const unsigned mm = (unsigned)(m < K ? m : K - 1);
    if (epi.fold) {  // uniform: v+ or v- of the unfolded axis at representative mm + roff
      const unsigned ma = mm + (unsigned)epi.roff;
      const unsigned mr = (unsigned)reflect_node((int)ma, epi.rn, epi.rper);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const double a = tb[xoff[e] + ma], b = tb[xoff[e] + mr];
        rx[e] = epi.fold == 1 ? a + b : a - b;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) rx[e] = tb[xoff[e] + mm];
    }
  };
  // contraction columns past K are zeroed at LDS-store time (after the MFMA block)
  auto store_chunk = [&](int buf, int c) {
    const bool ok = c * BK + tc < K;
    double* st = lds + buf * (TILE_T_NT + TILE_G);
    double* sg = st + TILE_T_NT;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kk = r0 + 4 * j;
      sg[kk * LDG + c0] = rg[2 * j];
      sg[kk * LDG + c0 + 64] = rg[2 * j + 1];
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) st[(tr + 16 * e) * LDT + tc] = ok ? rx[e] : 0.0;
  };

  d4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

  const int fr = lane & 15, fk = lane >> 4;
  auto compute_chunk = [&](int buf) {
    const double* st = lds + buf * (TILE_T_NT + TILE_G);
    const double* sg = st + TILE_T_NT;
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = st[(wm + 16 * i + fr) * LDT + ks * 4 + fk];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = sg[(ks * 4 + fk) * LDG + wn + 16 * j + fr];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  };

  if (nchunk > 0) {  // K = 0 (an empty antisymmetric block) stores zeros
    load_chunk(0);
    store_chunk(0, 0);
    __syncthreads();
    for (int c = 0; c + 1 < nchunk; ++c) {
      load_chunk(c + 1);
      // keep the LDS stores (which wait for the loads) after the whole MFMA block
      __builtin_amdgcn_sched_barrier(0);
      compute_chunk(c & 1);
      __builtin_amdgcn_sched_barrier(0);
      store_chunk((c + 1) & 1, c + 1);
      __syncthreads();
    }
    compute_chunk((nchunk - 1) & 1);
  }

#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long pp = p0 + wm + 16 * i + 4 * r + fk;
      if (pp >= P) continue;
      double* __restrict__ yrow = y + (size_t)pp * ldya;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int l = l0 + wn + 16 * j + fr;
        if (l >= L) continue;
        const double v = acc[i][j][r];
        if constexpr (EPI == EPI_STORE) yrow[l] = v;
        else if constexpr (EPI == EPI_DIVIDE)
          yrow[l] = v / spectral_den(epi.lx[l] + epi.ly[0] + epi.lz[0], epi.alpha, epi.b1, epi.b2);
        else if constexpr (EPI == EPI_SPECTRAL)
          yrow[l] = spectral_mul(v, epi.lx[l] + epi.ly[0] + epi.lz[0], epi);
        else if constexpr (EPI == EPI_UNFOLD) {  // column l holds o of representative l + roff
          const int lr = l + epi.roff, lm = reflect_node(lr, epi.rn, epi.rper);
          const double e = yrow[lr];
          yrow[lr] = e + v;
          if (lm != lr) yrow[lm] = e - v;
        } else yrow[l] += v;
      }
    }
}

// Compact reflection fold (see launch_fold_f64): blocks stride over the
// representatives, (p, r) when Q > 1 (threads over q), p when Q == 1 (threads over
// r); each reads x_r and x_R(r) once and writes v+ to row r and, unless r is its
// own reflection, v- to row nrep + r - off.
constexpr int FT = 256, FU = 4;
__global__ __launch_bounds__(FT) void fold_f64_kernel(const double* __restrict__ x, double* __restrict__ y, long P,
                                                      int n, long Q, int nrep, int per) {
  const int off = per ? 1 : 0;
  if (Q > 1) {
    const long rows = P * nrep;
    for (long row = blockIdx.x; row < rows; row += gridDim.x) {
      const long p = row / nrep;
      const int r = (int)(row - p * nrep), m = reflect_node(r, n, per);
      const double* __restrict__ xa = x + (size_t)(p * n + r) * Q;
      const double* __restrict__ xb = x + (size_t)(p * n + m) * Q;
      double* __restrict__ yp = y + (size_t)(p * n + r) * Q;
      double* __restrict__ ym = y + (size_t)(p * n + nrep + r - off) * Q;
      const bool minus = m != r;  // uniform over the block
      for (long q0 = threadIdx.x; q0 < Q; q0 += FT * FU) {
        double va[FU], vb[FU];
#pragma unroll
        for (int u = 0; u < FU; ++u) {
          const long q = q0 + (long)FT * u < Q ? q0 + (long)FT * u : Q - 1;
          va[u] = xa[q];
          vb[u] = xb[q];
        }
#pragma unroll
        for (int u = 0; u < FU; ++u) {
          const long q = q0 + (long)FT * u;
          if (q < Q) {
            yp[q] = va[u] + vb[u];
            if (minus) ym[q] = va[u] - vb[u];
          }
        }
      }
    }
  } else {
    for (long p = blockIdx.x; p < P; p += gridDim.x) {
      const double* __restrict__ xp = x + (size_t)p * n;
      double* __restrict__ yp = y + (size_t)p * n;
      for (int r0 = threadIdx.x; r0 < nrep; r0 += FT * FU) {
        double va[FU], vb[FU];
#pragma unroll
        for (int u = 0; u < FU; ++u) {
          const int r = r0 + FT * u < nrep ? r0 + FT * u : nrep - 1;
          va[u] = xp[r];
          vb[u] = xp[reflect_node(r, n, per)];
        }
#pragma unroll
        for (int u = 0; u < FU; ++u) {
          const int r = r0 + FT * u;
          if (r >= nrep) continue;
          yp[r] = va[u] + vb[u];
          if (reflect_node(r, n, per) != r) yp[nrep + r - off] = va[u] - vb[u];
        }
      }
    }
  }
}

}  // namespace f64k

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
// General form: Y[p][l][q] = sum_{m < K} A[l][m] X[p][m][q] for l < L, with the
// contracted axis of X of extent ldxa and the output axis of Y of extent ldya
// (batch strides ldxa Q and ldya Q); g[m * ldg + l] = A[l][m], padded so that
// whole 128 x 16 tiles stay inside (rows >= pad16(K), ldg >= pad128(L)).
hipError_t launch_mode_f64_part(const double* x, double* y, const double* g, int ldg, long P, int K, int L, long Q,
                                int ldxa, int ldya, int epi, const EpiArgs& ea, hipStream_t stream) {
  using namespace f64k;
  if (P <= 0 || Q <= 0 || L <= 0) return hipSuccess;
  if (K < 0 || K > ldxa || L > ldya) return hipErrorInvalidValue;
  if (Q > 1) {
    const long tiles_l = (L + BM - 1) / BM;
    const long tiles_q = (Q + BN - 1) / BN;
    const long ntiles = tiles_l * tiles_q * P;
    const long nbp = ((ntiles + 7) / 8) * 8;
    if (nbp > 0x7fffffffL) return hipErrorInvalidValue;
    dim3 grid((unsigned)nbp), block(NT_THREADS);
    switch (epi) {
      case EPI_STORE:
        mode_nn_f64<EPI_STORE><<<grid, block, 0, stream>>>(x, y, g, ldg, P, K, L, ldxa, ldya, Q, tiles_l, tiles_q,
                                                           ntiles, nbp, ea);
        break;
      case EPI_DIVIDE:
        mode_nn_f64<EPI_DIVIDE><<<grid, block, 0, stream>>>(x, y, g, ldg, P, K, L, ldxa, ldya, Q, tiles_l, tiles_q,
                                                            ntiles, nbp, ea);
        break;
      case EPI_SPECTRAL:
        mode_nn_f64<EPI_SPECTRAL><<<grid, block, 0, stream>>>(x, y, g, ldg, P, K, L, ldxa, ldya, Q, tiles_l,
                                                              tiles_q, ntiles, nbp, ea);
        break;
      case EPI_UNFOLD:
        mode_nn_f64<EPI_UNFOLD><<<grid, block, 0, stream>>>(x, y, g, ldg, P, K, L, ldxa, ldya, Q, tiles_l, tiles_q,
                                                            ntiles, nbp, ea);
        break;
      default:
        mode_nn_f64<EPI_ACCUM><<<grid, block, 0, stream>>>(x, y, g, ldg, P, K, L, ldxa, ldya, Q, tiles_l, tiles_q,
                                                           ntiles, nbp, ea);
        break;
    }
  } else {
    const long tiles_l = (L + BN - 1) / BN;
    const long tiles_p = (P + BM - 1) / BM;
    const long ntiles = tiles_l * tiles_p;
    const long nbp = ((ntiles + 7) / 8) * 8;
    if (nbp > 0x7fffffffL) return hipErrorInvalidValue;
    dim3 grid((unsigned)nbp), block(NT_THREADS);
    switch (epi) {
      case EPI_STORE:
        mode_nt_f64<EPI_STORE><<<grid, block, 0, stream>>>(x, y, g, ldg, P, K, L, ldxa, ldya, tiles_l, ntiles, nbp,
                                                           ea);
        break;
      case EPI_DIVIDE:  // only reached for the x axis with ny = nz = 1
        mode_nt_f64<EPI_DIVIDE><<<grid, block, 0, stream>>>(x, y, g, ldg, P, K, L, ldxa, ldya, tiles_l, ntiles, nbp,
                                                            ea);
        break;
      case EPI_SPECTRAL:
        mode_nt_f64<EPI_SPECTRAL><<<grid, block, 0, stream>>>(x, y, g, ldg, P, K, L, ldxa, ldya, tiles_l, ntiles,
                                                              nbp, ea);
        break;
      case EPI_UNFOLD:
        mode_nt_f64<EPI_UNFOLD><<<grid, block, 0, stream>>>(x, y, g, ldg, P, K, L, ldxa, ldya, tiles_l, ntiles, nbp,
                                                            ea);
        break;
      default:
        mode_nt_f64<EPI_ACCUM><<<grid, block, 0, stream>>>(x, y, g, ldg, P, K, L, ldxa, ldya, tiles_l, ntiles, nbp,
                                                           ea);
        break;
    }
  }
  return hipGetLastError();
}

hipError_t launch_fold_f64(const double* x, double* y, long P, int n, long Q, int nrep, int per, hipStream_t stream) {
  using namespace f64k;
  if (P <= 0 || Q <= 0 || n <= 0) return hipSuccess;
  if (nrep < 1 || nrep > n || 2 * nrep < n || x == y) return hipErrorInvalidValue;
  const long rows = Q > 1 ? P * nrep : P;
  const long grid = rows < 16384 ? rows : 16384;
  fold_f64_kernel<<<dim3((unsigned)grid), dim3(FT), 0, stream>>>(x, y, P, n, Q, nrep, per);
  return hipGetLastError();
}

// One dense mode product along `axis` of an (n0, n1, n2) array.
hipError_t launch_mode_f64(const double* x, double* y, const double* g, int ldg, const int dims[3], int axis, int epi,
                           const EpiArgs& ea, hipStream_t stream) {
  long P = 1, Q = 1;
  const int L = dims[axis];
  for (int a = 0; a < axis; ++a) P *= dims[a];
  for (int a = axis + 1; a < 3; ++a) Q *= dims[a];
  return launch_mode_f64_part(x, y, g, ldg, P, L, L, Q, L, L, epi, ea, stream);
}

}  // namespace semfd
