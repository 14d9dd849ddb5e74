// Internal declarations shared by the HIP translation units of the library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace semfd {

// EPI_SPECTRAL (FP64 kernels only): another multiplier than the divide (EpiArgs::kind)
// EPI_UNFOLD (FP64 kernels only): the output rows (NN) or columns (NT) are orbit
// representatives r of the output axis (EpiArgs::rn, rper) and the product is the
// antisymmetric part o: out[r] = e + o, out[R(r)] = e - o with e = out[r] as stored
// by the symmetric block before (R(r) == r: out[r] only)
enum { EPI_STORE = 0, EPI_DIVIDE = 1, EPI_ACCUM = 2, EPI_SPECTRAL = 3, EPI_UNFOLD = 4 };

// Arguments of the fused epilogues.
//   EPI_DIVIDE: out = acc / (alpha + b1 L + b2 L^2),  L = lx[row] + ly[col / nz] + lz[col % nz]
//               (Helmholtz: b1 = 1, b2 = 0; the Cahn-Hilliard operator a + m dt eps L^2:
//               b1 = 0, b2 = m dt eps)
//   EPI_ACCUM : out += acc
struct EpiArgs {
  const double* lx = nullptr;
  const double* ly = nullptr;
  const double* lz = nullptr;
  double alpha = 0.0, b1 = 1.0, b2 = 0.0;
  long nz = 1;
  // multiplier of EPI_SPECTRAL: SPECTRAL_EXP = exp(-param (L + alpha)),
  // SPECTRAL_POWER = (L + alpha)^(-param); EPI_DIVIDE divides by
  // alpha + b1 L + b2 L^2
  int kind = 0;
  double param = 0.0;
  // reflection split (FP64 kernels): fold = 1 / 2 reads the contracted axis (of
  // extent rn, periodic rper, x unfolded) as v+_r = x_r + x_R(r) / v-_r = x_r - x_R(r)
  // with r = m + roff for m < K; EPI_UNFOLD reflects the output axis (extent rn,
  // periodic rper) with output row / column l at representative r = l + roff
  int fold = 0;
  int rn = 0, rper = 0, roff = 0;
};
constexpr int SPECTRAL_EXP = 1, SPECTRAL_POWER = 2;

// Reflection of node r on an axis of n nodes: n - 1 - r, or (n - r) mod n periodic.
__host__ __device__ inline int reflect_node(int r, int n, int per) { return per ? (n - r) % n : n - 1 - r; }

// Denominator of the spectral divide, FP64.
__host__ __device__ inline double spectral_den(double lam, double alpha, double b1, double b2) {
  return alpha + lam * (b1 + b2 * lam);
}

// v times the multiplier of the EPI_SPECTRAL epilogue at eigenvalue sum lam.
__device__ inline double spectral_mul(double v, double lam, const EpiArgs& e) {
  if (e.kind == SPECTRAL_EXP) return v * exp(-e.param * (lam + e.alpha));
  return v * pow(fmax(lam + e.alpha, 0.0), -e.param);  // SPECTRAL_POWER; L >= 0 up to rounding
}

// One FP64 mode product along `axis` of a row-major (dims[0], dims[1], dims[2])
// array: y[.., l, ..] = sum_m A[l][m] x[.., m, ..] with g[m * ldg + l] = A[l][m]
// (g zero-padded to a multiple of 128 in both dimensions).
hipError_t launch_mode_f64(const double* x, double* y, const double* g, int ldg, const int dims[3], int axis, int epi,
                           const EpiArgs& ea, hipStream_t stream);
// General block form: Y[p][l][q] = sum_{m < K} A[l][m] X[p][m][q] for l < L, the
// contracted axis of X of extent ldxa, the output axis of Y of extent ldya (batch
// strides ldxa Q, ldya Q); g rows >= pad16(K), ldg >= pad128(L).  K = 0 stores zeros.
// ea.fold reads X as the v+ / v- of its unfolded axis; EPI_UNFOLD writes e +- o.
hipError_t launch_mode_f64_part(const double* x, double* y, const double* g, int ldg, long P, int K, int L, long Q,
                                int ldxa, int ldya, int epi, const EpiArgs& ea, hipStream_t stream);
// Compact reflection fold of X[p][i][q] along i (n nodes): Y[p][r] = X[p][r] + X[p][R(r)]
// for the nrep representatives, then Y[p][nrep + j] = X[p][r] - X[p][R(r)] for the
// n - nrep representatives r = j + off that are not their own reflection
// (off = 1 periodic, 0 otherwise): Y has n rows like X.
hipError_t launch_fold_f64(const double* x, double* y, long P, int n, long Q, int nrep, int per, hipStream_t stream);

// ---- low-precision rotating mode products (mode_lp.hip) ----
enum { LP_F32 = 1, LP_BF16 = 2, LP_BF16X3 = 3 };

// Epilogue arguments: divide by alpha + b1 L + b2 L^2 with L = l0[l] + l1[a] +
// l2[b] (third forward pass), or accumulate into FP64 (first = 1: u = delta)
// recording norms[0] = max|delta|, norms[1] = max|u| (bit patterns, atomic max;
// skipped when norms is null).
struct EpiLP {
  const double* l0 = nullptr;
  const double* l1 = nullptr;
  const double* l2 = nullptr;
  double alpha = 0.0, b1 = 1.0, b2 = 0.0;
  int first = 0;
  unsigned long long* norms = nullptr;
};

// One pass  Y[l][a][b] = sum_k F[l][k] X[a][b][k]:
//   x: input rows (P = A*B rows of K elements, row pitch ldx), kind in_kind
//      (0 FP64, 1 FP32, 2 BF16 bits);
//   y: output (L, A, B) with row pitch ldy, kind out_kind (1 FP32, 2 BF16, 0 FP64
//      accumulate);
//   f_hi / f_lo: factor [l][k] (FP32 or BF16 bits), padded with zeros to ldf
//      columns and to a multiple of 128 rows.
// The direct-to-LDS kernels (mode_dma.hip) take BF16 operands only: split-BF16
// operands are two planes, the second xplane / yplane / fplane elements after
// the first (f_lo unused).
// Output column layouts of the BF16 passes (mode_dma.hip): plain, split mode
// layout (symmetric block, then antisymmetric from column bpad), folded pairs.
enum { COL_PLAIN = 0, COL_SPLIT = 1, COL_FOLD = 2 };

struct LpPass {
  int mode = LP_BF16;
  const void* x = nullptr;
  int ldx = 0;
  long P = 0;
  int K = 0;
  void* y = nullptr;
  int ldy = 0;
  int A = 0, B = 0, L = 0;
  const void* f_hi = nullptr;
  const void* f_lo = nullptr;
  int ldf = 0;
  int in_kind = 0, out_kind = 0, epi_kind = EPI_STORE;
  long xplane = 0, yplane = 0, fplane = 0;
  EpiLP epi;
  // BF16 passes only: a second contraction block (K2 > 0): its l-tiles read factor
  // rows from frow2 (>= L rounded up to 256) and tensor k in [koff2, koff2 + K2),
  // and write L2 output rows after the L of block 1 (K, L: block 1)
  int K2 = 0, koff2 = 0, frow2 = 0, L2 = 0;
  // output column layout (COL_*) and the b axis: COL_SPLIT: bsym symmetric modes,
  // antisymmetric from column bpad; COL_FOLD: bsym = orbit representatives of the
  // b axis (length bn, periodic bper), v+ at column r, v- at bpad + r
  int col = COL_PLAIN;
  int bsym = 0, bpad = 0, bn = 0, bper = 0;
  // tuned launch shapes: FP32 factor-tile rows (128, 96, 64, 32; 0 = by rule);
  // BF16 tile order: groups of g p-strips step through the l-tiles together
  // (g = 1: every l-tile of one p-strip in a row); tile_group = g launches one
  // block per tile, DMA_PERSIST + g one block per CU looping over the tiles
  int tile_rows = 0;
  int tile_group = 1;
};
constexpr int DMA_PERSIST = 16;
// FP32 passes (mode_lp.hip): mode LP_F32, in_kind 0 or 1, out_kind 1 or 0 (accumulate).
hipError_t launch_mode_lp(const LpPass& ps, hipStream_t stream);

// One FP32 pass of one solve inside a batched (persistent) launch: the fields of
// LpPass plus the tile bookkeeping.  Descriptor i owns tiles [tile0, tile0 +
// tiles_l * ceil(P / 128)) of the launch's global tile numbering (ascending
// tile0); sid indexes the launch's per-solve active flags.
struct LpDesc {
  const void* x = nullptr;
  void* y = nullptr;
  const void* f = nullptr;  // FP32 factor [l][k], pitch ldf
  EpiLP epi;
  long P = 0;
  long tile0 = 0;
  int ldx = 0, K = 0, ldy = 0, A = 0, B = 0, L = 0, ldf = 0;
  int tiles_l = 0;
  int sid = 0;
};
// Persistent FP32 launch over nd descriptors (device array) with tile_rows in
// {128, 96, 64, 32} (block tile tile_rows x 128), grid blocks striding over
// total_tiles; active: device array of per-solve flags.
hipError_t launch_mode_f32_batch(int in_kind, int out_kind, int epi, int tile_rows, const LpDesc* descs, int nd,
                                 long total_tiles, const int* active, int grid, hipStream_t stream);
int lp_batch_blocks_per_cu(int tile_rows);

// ---- BF16 / split-BF16 passes with direct global -> LDS loads (mode_dma.hip) ----
// Requirements: in_kind 2, ldx, ldy and ldf multiples of 8, each contraction
// block inside the tensor pitch and the factor pitch rounded to 32; tensor pitch
// padding holds finite values; factor zero outside its blocks.  Outputs: BF16
// planes (out_kind 2, any column layout, STORE or DIVIDE) or FP32 (out_kind 1,
// COL_PLAIN, STORE).  Padding columns receive finite values.
bool dma_supported(const LpPass& ps);
hipError_t launch_mode_dma(const LpPass& ps, hipStream_t stream);
// Reflection split of one axis: nrep orbit representatives (v+ at columns
// [0, pad), v- at [pad, 2 pad) of a folded row), reflection n - 1 - r or, per,
// (n - r) mod n.
struct FoldAxis {
  int nrep = 0, pad = 0, per = 0;
};
// FP64 array (rows dims[0]*dims[1], pitch dims[2]) -> BF16 hi (+ lo plane plane_o
// elements later when split) with pitch ldo, padding zeroed; fold != null: the rows
// folded along z first.
hipError_t launch_to_lowp(const double* f, void* out, long plane_o, int split, const int dims[3], int ldo,
                          const FoldAxis* fold, hipStream_t stream);
// BF16 (split) rows of pitch ldi -> the same rows folded along z, pitch ldo.
hipError_t launch_fold_lowp(const void* in, long plane_i, int ldi, void* out, long plane_o, int ldo, int split,
                            const int dims[3], const FoldAxis& fold, hipStream_t stream);
// Weighted inner products an unfold with first = 1 forms as it writes u: per-block
// partial sums of <r, u>_M and <u, q>_M (mass weight mx_i my_j mz_l of node (i, j, l))
// into partial[2 b] and partial[2 b + 1], b < blocks (the grid of such a launch).
struct UnfoldDot {
  const double* r = nullptr;
  const double* q = nullptr;
  const double *mx = nullptr, *my = nullptr, *mz = nullptr;
  double* partial = nullptr;
  int blocks = 0;
};
// u (+)= the correction d (FP32, every axis in folded node form: e rows then o
// rows, pitch ldd for z''), see unfold_accum_kernel; dot (first = 1 only): also
// the partial sums of UnfoldDot.
hipError_t launch_unfold_accum(const float* d, int ldd, double* u, const int dims[3], const FoldAxis fold[3],
                               int first, unsigned long long* norms, hipStream_t stream,
                               const UnfoldDot* dot = nullptr);

// Generalised nodal residual  r = cf f - cd d - ch (H_x + H_y + H_z) v  with banded
// H rows hb[a][g * (2k+1) + d] = H_a(g, g - k + d), FP64 arithmetic.
//   f == nullptr: the f term is absent;  d == nullptr: d is v itself.
//   Helmholtz residual f - alpha u - H u: (v = u, f, d = null, cf = 1, cd = alpha, ch = 1).
// r is written with row pitch ldr >= dims[2] as FP64 (r_kind 0), FP32 (1), BF16
// (2) or split BF16 (3: hi plane, lo plane rplane elements later); the pitch
// padding [dims[2], ldr) is written with zeros.  r must not alias v.
struct ResidualArgs {
  const double* v = nullptr;
  const double* f = nullptr;
  const double* d = nullptr;
  // optional per-node weight of the d term, cd * (wa + wt) * (d or v); FP64 output
  // (r_kind 0) of the single launch only
  const double* wt = nullptr;
  double wa = 0.0;
  void* r = nullptr;
  int r_kind = 0;
  int ldr = 0;
  long rplane = 0;
  double cf = 1.0, cd = 0.0, ch = 1.0;
  int periodic = 0;  // bit a set: axis a is periodic (its neighbours wrap around)
  // weighted march only (wt set, k <= 8, FP64 output): also the per-block partial
  // sums of <v, r>_M = sum Mx_i My_j Mz_l v r, written to dot_partial[2 b] for
  // block b of the launch (residual_march_blocks blocks); dot_mass = the 1D masses
  double* dot_partial = nullptr;
  const double* dot_mass[3] = {nullptr, nullptr, nullptr};
};
// Blocks of the single-launch march for these dimensions and k (0 for k > 8,
// which takes the generic kernel).
long residual_march_blocks(const int dims[3], int k);
hipError_t launch_residual(const ResidualArgs& ra, const double* const hb[3], int k, const int dims[3],
                           hipStream_t stream);

// Residuals of many solves with the same k (1..8) in one launch.  Descriptor i
// (device array, ascending block0) owns blocks [block0, block0 + gx*gy*gz);
// active: device array of per-solve flags indexed by sid.
struct ResDesc {
  const double* v = nullptr;
  const double* f = nullptr;
  const double* d = nullptr;
  void* r = nullptr;
  const double* hx = nullptr;
  const double* hy = nullptr;
  const double* hz = nullptr;
  long rplane = 0;
  long block0 = 0;
  int ldr = 0, nx = 0, ny = 0, nz = 0, xchunk = 0, gx = 0, gy = 0, gz = 0;
  int sid = 0;
  double cf = 1.0, cd = 0.0, ch = 1.0;
  int per = 0;  // bit a set: axis a is periodic (neighbours wrap around)
};
// Fill the geometry and operands of one descriptor (block0 and sid are the
// caller's); false if k or the arguments are outside what the batch kernel takes.
bool residual_desc(const ResidualArgs& ra, const double* const hb[3], int k, const int dims[3], ResDesc* d);
hipError_t launch_residual_batch(int k, int r_kind, const ResDesc* descs, int nd, long total_blocks,
                                 const int* active, hipStream_t stream);

}  // namespace semfd
