// Variable coefficients: alpha u - Lap u + V(x) u = f (the paper's Schrodinger-
// equation section, eq. shrodinger) by preconditioned conjugate gradients with
// the fast-diagonalisation solve of (shift I - Lap) as the preconditioner; the
// paper takes shift = alpha + beta/2 for 0 <= V <= beta.
//
// Discrete form (GLL quadrature, nodal): A u = alpha u + H_3 u + V u = f, with
// H_3 = M_3^{-1} K_3.  A and P = shift I + H_3 are self-adjoint and positive in
// the M_3-weighted inner product <a, b> = sum M_3 a b, which the iteration uses
// throughout (the iterates of plain PCG on the symmetric weak form).
//
// One iteration on the GPU: q = A p (the matrix-free residual kernel with the
// per-node weight alpha + V, which for k <= 8 also sums <p, q> per block); u += a p
// and r -= a q fused with <r, r>;
// z = P^{-1} r (an FP64 FD solve, or a low-precision one); <r, z> (and <z, q>);
// p = z + b p.  With a BF16 preconditioner (reflection-split passes) the update
// also writes the new r folded along z in BF16, the input of the preconditioner's
// first pass, and the preconditioner's unfold into z forms <r, z> and <z, q>.  The weighted inner products are two-stage block reductions
// (fixed block count, partial sums added in a fixed order: deterministic); the
// mass weight of node (i, j, l) is Mx_i My_j Mz_l from the three 1D masses.
//
// With a low-precision preconditioner the operator P^{-1} varies slightly from
// one application to the next, so b uses the flexible (Polak-Ribiere) form
// <z_new, r_new - r_old> / <z_old, r_old> = -a <z_new, q> / <z_old, r_old>,
// which equals the classical <z_new, r_new> / <z_old, r_old> for a fixed
// preconditioner; the FP64 preconditioner uses the classical form.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <cstring>

#include "kernels.h"
#include "plan_internal.h"

namespace semfd {
namespace {

constexpr int DOT_BLOCKS = 4096, DOT_THREADS = 256, MAXDOT = 2;

inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < DOT_THREADS / 64; ++w) t += sh[w];
  __syncthreads();
  return t;  // valid in thread 0
}

// Partial sums of NDOT weighted products <a_d, b_d> per block, rows (i, j) strided
// over the blocks, the z line of a row over the threads.
template <int NDOT>
__global__ __launch_bounds__(DOT_THREADS) void mdot_partial(const double* __restrict__ a0,
                                                            const double* __restrict__ b0,
                                                            const double* __restrict__ a1,
                                                            const double* __restrict__ b1,
                                                            const double* __restrict__ mx,
                                                            const double* __restrict__ my,
                                                            const double* __restrict__ mz, int nx, int ny, int nz,
                                                            double* __restrict__ partial) {
  __shared__ double sh[DOT_THREADS / 64];
  double s0 = 0.0, s1 = 0.0;
  const long rows = (long)nx * ny;
  for (long row = blockIdx.x; row < rows; row += gridDim.x) {
    const int i = (int)(row / ny), j = (int)(row - (long)i * ny);
    const double mr = mx[i] * my[j];
    const size_t base = (size_t)row * nz;
    for (int l = threadIdx.x; l < nz; l += DOT_THREADS) {
      const double m = mr * mz[l];
      s0 += m * a0[base + l] * b0[base + l];
      if (NDOT > 1) s1 += m * a1[base + l] * b1[base + l];
    }
  }
  const double t0 = block_sum(s0, sh);
  if (threadIdx.x == 0) partial[(size_t)blockIdx.x * MAXDOT] = t0;
  if (NDOT > 1) {
    const double t1 = block_sum(s1, sh);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.x * MAXDOT + 1] = t1;
  }
}

// u += a p, r -= a q, and the partial sums of <r, r> (new r).
__global__ __launch_bounds__(DOT_THREADS) void pcg_update(double* __restrict__ u, double* __restrict__ r,
                                                          const double* __restrict__ p,
                                                          const double* __restrict__ q, double a,
                                                          const double* __restrict__ mx,
                                                          const double* __restrict__ my,
                                                          const double* __restrict__ mz, int nx, int ny, int nz,
                                                          double* __restrict__ partial) {
  __shared__ double sh[DOT_THREADS / 64];
  double s = 0.0;
  const long rows = (long)nx * ny;
  for (long row = blockIdx.x; row < rows; row += gridDim.x) {
    const int i = (int)(row / ny), j = (int)(row - (long)i * ny);
    const double mr = mx[i] * my[j];
    const size_t base = (size_t)row * nz;
    for (int l = threadIdx.x; l < nz; l += DOT_THREADS) {
      const size_t g = base + l;
      u[g] += a * p[g];
      const double rn = r[g] - a * q[g];
      r[g] = rn;
      s += mr * mz[l] * rn * rn;
    }
  }
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) partial[(size_t)blockIdx.x * MAXDOT] = t;
}

// The same update for a reflection-split BF16 preconditioner, which also writes
// the new r folded along z and rounded to BF16 (hi, and lo = r - hi when split),
// the input of the preconditioner's first pass: v+ = r_z + r_R(z) at column z,
// v- = r_z - r_R(z) at fpad + z for the nrep representatives z (the sums in FP64,
// then FP32, then BF16, as the conversion kernel of the FD application does),
// zeros in the rest of the row of pitch 2 fpad.  A thread takes a representative
// and its reflection (once for a fixed node).
template <int NS>
__global__ __launch_bounds__(DOT_THREADS) void pcg_update_fold(double* __restrict__ u, double* __restrict__ r,
                                                               const double* __restrict__ p,
                                                               const double* __restrict__ q, double a,
                                                               const double* __restrict__ mx,
                                                               const double* __restrict__ my,
                                                               const double* __restrict__ mz, int nx, int ny, int nz,
                                                               double* __restrict__ partial,
                                                               unsigned short* __restrict__ o, long plane_o, int nrep,
                                                               int fpad, int per) {
  __shared__ double sh[DOT_THREADS / 64];
  double s = 0.0;
  const long rows = (long)nx * ny;
  for (long row = blockIdx.x; row < rows; row += gridDim.x) {
    const int i = (int)(row / ny), j = (int)(row - (long)i * ny);
    const double mr = mx[i] * my[j];
    const size_t base = (size_t)row * nz;
    unsigned short* __restrict__ orow = o + (size_t)row * 2 * fpad;
    for (int zr = threadIdx.x; zr < fpad; zr += DOT_THREADS) {
      double vp = 0.0, vm = 0.0;
      if (zr < nrep) {
        const int zm = per ? (nz - zr) % nz : nz - 1 - zr;
        const size_t g0 = base + zr, g1 = base + zm;
        u[g0] += a * p[g0];
        const double r0 = r[g0] - a * q[g0];
        r[g0] = r0;
        s += mr * mz[zr] * r0 * r0;
        double r1 = r0;
        if (zm != zr) {
          u[g1] += a * p[g1];
          r1 = r[g1] - a * q[g1];
          r[g1] = r1;
          s += mr * mz[zm] * r1 * r1;
        }
        vp = r0 + r1;
        vm = r0 - r1;
      }
      const float fp = (float)vp, fm = (float)vm;
      const __bf16 hp = (__bf16)fp, hm = (__bf16)fm;
      orow[zr] = __builtin_bit_cast(unsigned short, hp);
      orow[fpad + zr] = __builtin_bit_cast(unsigned short, hm);
      if (NS == 2) {
        orow[plane_o + zr] = __builtin_bit_cast(unsigned short, (__bf16)(fp - (float)hp));
        orow[plane_o + fpad + zr] = __builtin_bit_cast(unsigned short, (__bf16)(fm - (float)hm));
      }
    }
  }
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) partial[(size_t)blockIdx.x * MAXDOT] = t;
}

// Fixed-order sum of the block partials: out[d] = sum_b partial[b][d].
__global__ __launch_bounds__(DOT_THREADS) void mdot_final(const double* __restrict__ partial, int nblocks, int ndot,
                                                          double* __restrict__ out) {
  __shared__ double sh[DOT_THREADS / 64];
  for (int d = 0; d < ndot; ++d) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += DOT_THREADS) s += partial[(size_t)b * MAXDOT + d];
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) out[d] = t;
  }
}

// Partial maxima of V per block (a NaN or Inf gives +Inf, so the caller sees a
// non-finite shift), then their maximum: the default shift alpha + max(V) / 2.
__global__ __launch_bounds__(DOT_THREADS) void vmax_partial(const double* __restrict__ v, size_t n,
                                                            double* __restrict__ partial) {
  __shared__ double sh[DOT_THREADS / 64];
  double m = -INFINITY;
  for (size_t g = (size_t)blockIdx.x * DOT_THREADS + threadIdx.x; g < n; g += (size_t)gridDim.x * DOT_THREADS) {
    const double x = v[g];
    m = fabs(x) <= DBL_MAX ? fmax(m, x) : INFINITY;
  }
  for (int s = 32; s >= 1; s >>= 1) m = fmax(m, __shfl_xor(m, s));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = sh[0];
    for (int w = 1; w < DOT_THREADS / 64; ++w) t = fmax(t, sh[w]);
    partial[(size_t)blockIdx.x * MAXDOT] = t;
  }
}

__global__ __launch_bounds__(DOT_THREADS) void default_shift(const double* __restrict__ partial, int nblocks,
                                                             double alpha, double* __restrict__ out) {
  __shared__ double sh[DOT_THREADS / 64];
  double m = -INFINITY;
  for (int b = threadIdx.x; b < nblocks; b += DOT_THREADS) m = fmax(m, partial[(size_t)b * MAXDOT]);
  for (int s = 32; s >= 1; s >>= 1) m = fmax(m, __shfl_xor(m, s));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = sh[0];
    for (int w = 1; w < DOT_THREADS / 64; ++w) t = fmax(t, sh[w]);
    out[0] = alpha + 0.5 * t;
  }
}

// p = z + b p
__global__ __launch_bounds__(256) void pcg_direction(double* __restrict__ p, const double* __restrict__ z, double b,
                                                     size_t n) {
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (size_t)gridDim.x * blockDim.x)
    p[g] = z[g] + b * p[g];
}

struct PcgWork {
  double *r, *z, *p, *q, *partial, *out;
};

// block partials: the dot kernels' DOT_BLOCKS, or the operator march's blocks
size_t partial_slots(const sem_plan* p) {
  return (size_t)std::max<long>(DOT_BLOCKS, residual_march_blocks(p->dims, p->k));
}

size_t pcg_need(const sem_plan* p) {
  return 4 * align256(p->N * sizeof(double)) + align256(partial_slots(p) * MAXDOT * sizeof(double)) + 256;
}

int dot_blocks(const sem_plan* p) {
  const long rows = (long)p->dims[0] * p->dims[1];
  return (int)(rows < DOT_BLOCKS ? rows : DOT_BLOCKS);
}

// <a0, b0> (and <a1, b1>) into host h[0..ndot)
hipError_t mdot(sem_plan* p, const PcgWork& w, int ndot, const double* a0, const double* b0, const double* a1,
                const double* b1, double* h) {
  const int nb = dot_blocks(p);
  if (ndot == 1)
    mdot_partial<1><<<nb, DOT_THREADS, 0, p->stream>>>(a0, b0, a0, b0, p->d_mass[0], p->d_mass[1], p->d_mass[2],
                                                       p->dims[0], p->dims[1], p->dims[2], w.partial);
  else
    mdot_partial<2><<<nb, DOT_THREADS, 0, p->stream>>>(a0, b0, a1, b1, p->d_mass[0], p->d_mass[1], p->d_mass[2],
                                                       p->dims[0], p->dims[1], p->dims[2], w.partial);
  mdot_final<<<1, DOT_THREADS, 0, p->stream>>>(w.partial, nb, ndot, w.out);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(h, w.out, ndot * sizeof(double), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  return e;
}

}  // namespace
}  // namespace semfd

using namespace semfd;

extern "C" {

sem_status sem_pcg_workspace_bytes(const sem_plan* p, size_t* bytes) {
  if (!p || !bytes) return set_error(SEM_EINVAL, "sem_pcg_workspace_bytes: null argument");
  *bytes = pcg_need(p);
  return SEM_OK;
}

sem_status sem_pcg_solve(sem_plan* p, const double* v, double shift, sem_prec prec, double tol, int max_iter,
                         const double* f, double* u, void* work, size_t work_bytes, int* iters, double* relres,
                         double* shift_used) {
  if (iters) *iters = 0;
  if (shift_used) *shift_used = NAN;
  if (relres) *relres = NAN;
  if (!p || !v || !f || !u || !work) return set_error(SEM_EINVAL, "sem_pcg_solve: null argument");
  if (u == f || u == v) return set_error(SEM_EINVAL, "sem_pcg_solve: u must not alias f or V");
  if (std::isnan(shift) || std::isinf(shift)) return set_error(SEM_EINVAL, "sem_pcg_solve: shift must be finite");
  if (!(tol >= 0.0) || !std::isfinite(tol) || max_iter < 1)
    return set_error(SEM_EINVAL, "sem_pcg_solve: invalid tol or max_iter");
  if (prec != SEM_F64 && prec != SEM_F32 && prec != SEM_BF16 && prec != SEM_BF16X3)
    return set_error(SEM_EINVAL, "sem_pcg_solve: unknown precision");
  if (work_bytes < pcg_need(p) || ((uintptr_t)work & 255))
    return set_error(SEM_EINVAL, "sem_pcg_solve: workspace too small or not 256-byte aligned");
  const size_t n = p->N;
  const size_t vb = align256(n * sizeof(double));
  char* wb = (char*)work;
  PcgWork w{(double*)wb, (double*)(wb + vb), (double*)(wb + 2 * vb), (double*)(wb + 3 * vb),
            (double*)(wb + 4 * vb), (double*)(wb + 4 * vb + align256(partial_slots(p) * MAXDOT * sizeof(double)))};

  hipError_t e;
  double h[2];
  if (!(shift > 0.0)) {
    // default: the paper's alpha + beta / 2 with beta = max(V)
    const int nb0 = dot_blocks(p);
    vmax_partial<<<nb0, DOT_THREADS, 0, p->stream>>>(v, n, w.partial);
    default_shift<<<1, DOT_THREADS, 0, p->stream>>>(w.partial, nb0, p->alpha, w.out);
    if ((e = hipGetLastError()) != hipSuccess ||
        (e = hipMemcpyAsync(h, w.out, sizeof(double), hipMemcpyDeviceToHost, p->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(p->stream)) != hipSuccess)
      return hip_fail(e, "sem_pcg_solve: default shift");
    shift = h[0];
    if (!std::isfinite(shift)) return set_error(SEM_ENONFINITE, "sem_pcg_solve: non-finite potential");
    if (!(shift > 0.0)) return set_error(SEM_EINVAL, "sem_pcg_solve: default shift alpha + max(V)/2 is not > 0");
  }
  if (shift_used) *shift_used = shift;
  // preconditioner z = (shift I + H_3)^{-1} r
  const Spectral sp{shift, 1.0, 0.0};
  LpWork lw;
  double* tmp64 = nullptr;
  if (prec == SEM_F64) {
    void* ws = nullptr;
    sem_status st = plan_workspace(p, workspace_need(p, SEM_F64), &ws);
    if (st != SEM_OK) return st;
    tmp64 = (double*)ws;
  } else {
    sem_status st = lp_prepare(p, prec, &lw);
    if (st != SEM_OK) return st;
  }
  // BF16 modes: after the first application (from r = f), the update writes the
  // folded BF16 r itself and the application starts at its first pass
  // and the unfold into z forms <r, z>_M and <z, q>_M as it writes z
  FoldAxis fz;
  bool fold_update = false;
  UnfoldDot ud;
  if (prec == SEM_BF16 || prec == SEM_BF16X3) {
    FoldAxis fa[3];
    lp_fold_axes(p, fa);
    fz = fa[2];
    fold_update = lp_fold_pitch_z(p) == 2 * fz.pad;
    ud.r = w.r;
    ud.q = w.q;
    ud.mx = p->d_mass[0];
    ud.my = p->d_mass[1];
    ud.mz = p->d_mass[2];
    ud.partial = w.partial;
    ud.blocks = (int)std::min<long>((long)fa[0].nrep * fa[1].nrep, DOT_BLOCKS);
  }
  auto precondition = [&]() -> hipError_t {
    return prec == SEM_F64 ? fd64(p, sp, w.r, w.z, tmp64) : lp_fd(p, lw, sp, w.r, w.z, 1, nullptr);
  };
  // q = A p = (alpha + V) p + H_3 p
  ResidualArgs ra;
  ra.periodic = p->per_mask;
  ra.v = w.p;
  ra.f = nullptr;
  ra.wt = v;
  ra.wa = p->alpha;
  ra.r = w.q;
  ra.r_kind = 0;
  ra.ldr = p->dims[2];
  ra.cf = 0.0;
  ra.cd = -1.0;
  ra.ch = -1.0;
  const double* hb[3] = {p->d_hb[0], p->d_hb[1], p->d_hb[2]};
  const int nb = dot_blocks(p);
  const unsigned gdir = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
  // <p, q> from the operator launch itself (k <= 8: the march kernel)
  const long fused_blocks = residual_march_blocks(p->dims, p->k);
  if (fused_blocks > 0) {
    ra.dot_partial = w.partial;
    for (int a = 0; a < 3; ++a) ra.dot_mass[a] = p->d_mass[a];
  }

  // u = 0, r = f
  if ((e = hipMemsetAsync(u, 0, n * sizeof(double), p->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(w.r, f, n * sizeof(double), hipMemcpyDeviceToDevice, p->stream)) != hipSuccess ||
      (e = mdot(p, w, 1, f, f, nullptr, nullptr, h)) != hipSuccess)
    return hip_fail(e, "sem_pcg_solve: start");
  const double fn2 = h[0];
  if (!std::isfinite(fn2)) return set_error(SEM_ENONFINITE, "sem_pcg_solve: non-finite right-hand side");
  if (fn2 == 0.0) {
    if (relres) *relres = 0.0;
    return SEM_OK;
  }
  if ((e = precondition()) != hipSuccess || (e = mdot(p, w, 1, w.r, w.z, nullptr, nullptr, h)) != hipSuccess ||
      (e = hipMemcpyAsync(w.p, w.z, n * sizeof(double), hipMemcpyDeviceToDevice, p->stream)) != hipSuccess)
    return hip_fail(e, "sem_pcg_solve: first preconditioner application");
  double rz = h[0];
  double rel = 1.0;
  for (int it = 1; it <= max_iter; ++it) {
    if ((e = launch_residual(ra, hb, p->k, p->dims, p->stream)) != hipSuccess)
      return hip_fail(e, "sem_pcg_solve: operator");
    if (fused_blocks > 0) {
      mdot_final<<<1, DOT_THREADS, 0, p->stream>>>(w.partial, (int)fused_blocks, 1, w.out);
      if ((e = hipGetLastError()) != hipSuccess ||
          (e = hipMemcpyAsync(h, w.out, sizeof(double), hipMemcpyDeviceToHost, p->stream)) != hipSuccess ||
          (e = hipStreamSynchronize(p->stream)) != hipSuccess)
        return hip_fail(e, "sem_pcg_solve: <p, q>");
    } else if ((e = mdot(p, w, 1, w.p, w.q, nullptr, nullptr, h)) != hipSuccess) {
      return hip_fail(e, "sem_pcg_solve: <p, q>");
    }
    const double pq = h[0];
    if (!std::isfinite(pq) || !std::isfinite(rz)) return set_error(SEM_ENONFINITE, "sem_pcg_solve: non-finite iterate");
    if (!(pq > 0.0) || !(rz > 0.0))
      return set_error(SEM_ENOCONV, "sem_pcg_solve: operator or preconditioner not positive definite");
    const double a = rz / pq;
    if (fold_update) {
      // the update also writes the preconditioner's folded BF16 input
      if (prec == SEM_BF16X3)
        pcg_update_fold<2><<<nb, DOT_THREADS, 0, p->stream>>>(
            u, w.r, w.p, w.q, a, p->d_mass[0], p->d_mass[1], p->d_mass[2], p->dims[0], p->dims[1], p->dims[2],
            w.partial, (unsigned short*)lw.t1, lw.tplane, fz.nrep, fz.pad, fz.per);
      else
        pcg_update_fold<1><<<nb, DOT_THREADS, 0, p->stream>>>(
            u, w.r, w.p, w.q, a, p->d_mass[0], p->d_mass[1], p->d_mass[2], p->dims[0], p->dims[1], p->dims[2],
            w.partial, (unsigned short*)lw.t1, lw.tplane, fz.nrep, fz.pad, fz.per);
      lw.input_in_t1 = true;
      lw.unfold_dot = &ud;
    } else {
      pcg_update<<<nb, DOT_THREADS, 0, p->stream>>>(u, w.r, w.p, w.q, a, p->d_mass[0], p->d_mass[1], p->d_mass[2],
                                                     p->dims[0], p->dims[1], p->dims[2], w.partial);
    }
    mdot_final<<<1, DOT_THREADS, 0, p->stream>>>(w.partial, nb, 1, w.out);
    if ((e = hipGetLastError()) != hipSuccess ||
        (e = hipMemcpyAsync(h, w.out, sizeof(double), hipMemcpyDeviceToHost, p->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(p->stream)) != hipSuccess)
      return hip_fail(e, "sem_pcg_solve: update");
    rel = std::sqrt(h[0] / fn2);
    if (iters) *iters = it;
    if (relres) *relres = rel;
    if (!std::isfinite(rel)) return set_error(SEM_ENONFINITE, "sem_pcg_solve: non-finite residual");
    if (rel <= tol) return SEM_OK;
    if (it == max_iter) break;
    if ((e = precondition()) != hipSuccess) return hip_fail(e, "sem_pcg_solve: preconditioner");
    double b;
    if (prec == SEM_F64) {
      if ((e = mdot(p, w, 1, w.r, w.z, nullptr, nullptr, h)) != hipSuccess) return hip_fail(e, "sem_pcg_solve: dot");
      b = h[0] / rz;
      rz = h[0];
    } else {
      if (lw.unfold_dot) {  // partials from the preconditioner's unfold
        mdot_final<<<1, DOT_THREADS, 0, p->stream>>>(w.partial, ud.blocks, 2, w.out);
        if ((e = hipGetLastError()) != hipSuccess ||
            (e = hipMemcpyAsync(h, w.out, 2 * sizeof(double), hipMemcpyDeviceToHost, p->stream)) != hipSuccess ||
            (e = hipStreamSynchronize(p->stream)) != hipSuccess)
          return hip_fail(e, "sem_pcg_solve: dot");
      } else if ((e = mdot(p, w, 2, w.r, w.z, w.z, w.q, h)) != hipSuccess) {
        return hip_fail(e, "sem_pcg_solve: dot");
      }
      b = -a * h[1] / rz;
      rz = h[0];
    }
    pcg_direction<<<gdir, 256, 0, p->stream>>>(w.p, w.z, b, n);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "sem_pcg_solve: direction");
  }
  if (tol > 0) return set_error(SEM_ENOCONV, "sem_pcg_solve: tolerance not met within max_iter");
  return SEM_OK;
}

}  // extern "C"
