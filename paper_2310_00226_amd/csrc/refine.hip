// Mixed-precision solve with FP64 iterative refinement.
//
//   u = 0, r = f
//   repeat: delta = S_3 [ (F_3 r) ./ (Lambda3D + alpha) ]   (mode products in low precision)
//           u += delta                                      (FP64, fused into the last pass)
//           r  = f - M_3^{-1} A u                           (FP64 matrix-free residual)
//   until ||delta||_inf <= tol ||u||_inf, or the observed contraction of the
//   updates predicts that the remaining error is below that (refine_converged).
// The low-precision solve is eq. 3D-Poisson of the paper (Sec. 2.4) with its
// mode products rounded to FP32 / BF16; the refinement around it is not in the
// paper (its single-precision runs plateau without it, Table 10).
//
// Each low-precision solve is six rotating mode products:
//   (x,y,z) -z-> (z,x,y) -y-> (y,z,x) -x,divide-> (x,y,z) -z-> (z,x,y) -y-> (y,z,x) -x-> u
// Intermediates live in the workspace with their contiguous axis padded to a
// multiple of 8 elements (16-byte rows for BF16).  FP32 runs the register-staged
// kernels of mode_lp.hip; BF16 and split BF16 run the direct-to-LDS kernels of
// mode_dma.hip, with every operand in BF16 planes (split: a hi plane and a lo
// plane): the right-hand side is converted once, the residual is written in that
// format directly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "kernels.h"
#include "plan_internal.h"

namespace semfd {

namespace {

inline int pad8(int n) { return (n + 7) / 8 * 8; }
inline int pad256(int n) { return (n + 255) / 256 * 256; }
// Row pitch of the low-precision intermediates.  FP32 rows are padded to 8
// elements.  BF16 rows (streamed into LDS as 64-byte chunks) are padded to 32
// elements, so that every chunk sits inside one 128-byte cache line: with an
// unaligned pitch half of the chunks straddle two lines, which measured 6-12%
// slower passes at n = 999.
inline int lp_pitch(int n, sem_prec prec) { return prec == SEM_F32 ? pad8(n) : (n + 31) / 32 * 32; }

unsigned short host_f2bf(float f) {
  unsigned u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
float host_bf2f(unsigned short b) {
  unsigned u = ((unsigned)b) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// bytes per element of the intermediates (split BF16: two 2-byte planes)
size_t lp_elem(sem_prec prec) { return prec == SEM_BF16 ? 2 : 4; }
bool lp_split(sem_prec prec) { return prec == SEM_BF16X3; }

// largest of the three rotated padded layouts (z,x,y'), (y,z,x'), (x,y,z')
size_t lp_tmp_elems(const sem_plan* p, sem_prec prec) {
  const size_t nx = p->dims[0], ny = p->dims[1], nz = p->dims[2];
  return std::max({nz * nx * (size_t)lp_pitch((int)ny, prec), ny * nz * (size_t)lp_pitch((int)nx, prec),
                   nx * ny * (size_t)lp_pitch((int)nz, prec)});
}

// residual buffer of the refinement: (nx, ny, pitch(nz)) in the intermediate type
size_t lp_r_elems(const sem_plan* p, sem_prec prec) {
  return (size_t)p->dims[0] * p->dims[1] * lp_pitch(p->dims[2], prec);
}
size_t lp_r_bytes(const sem_plan* p, sem_prec prec) {
  return ((lp_r_elems(p, prec) * lp_elem(prec) + 255) / 256) * 256;
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

}  // namespace

size_t workspace_need(const sem_plan* p, sem_prec prec) {
  const size_t n = p->N;
  switch (prec) {
    case SEM_F64:
      return ((n * sizeof(double) + 255) / 256) * 256;
    case SEM_F32:
    case SEM_BF16:
    case SEM_BF16X3: {
      const size_t r = lp_r_bytes(p, prec);
      const size_t t = ((lp_tmp_elems(p, prec) * lp_elem(prec) + 255) / 256) * 256;
      return r + 2 * t + 256;
    }
    default:
      return 0;
  }
}

void release_lowp(sem_plan* p) {
  for (int a = 0; a < 3; ++a)
    for (int d = 0; d < 2; ++d) {
      (void)hipFree(p->lp_f32[a][d]);
      (void)hipFree(p->lp_hi[a][d]);  // lp_lo points into the same allocation
      p->lp_f32[a][d] = p->lp_hi[a][d] = p->lp_lo[a][d] = nullptr;
    }
  p->lp_ready = 0;
}

// Low-precision copies of the factors, layout [l][k] (row l = output mode,
// contraction k contiguous), zero-padded to pitch ld = pad256(n): FP32 with
// ld + 96 rows (whole tiles of 128, 96, 64 or 32 rows stay inside), and BF16 hi
// followed by BF16 lo = bf16(v - hi) with ld rows each in one allocation
// (lp_lo = lp_hi + ld * ld elements).
static sem_status ensure_lowp(sem_plan* p) {
  if (p->lp_ready) return SEM_OK;
  for (int a = 0; a < 3; ++a) {
    const int n = p->dims[a], ld = pad256(n);
    const size_t plane = (size_t)ld * ld;
    p->lp_ld[a] = ld;
    for (int d = 0; d < 2; ++d) {
      const std::vector<double>& M = d == 0 ? p->ax[a].F : p->ax[a].S;
      std::vector<float> f32(plane + 96 * (size_t)ld, 0.0f);
      std::vector<unsigned short> hl(2 * plane, 0);
      for (int l = 0; l < n; ++l)
        for (int k = 0; k < n; ++k) {
          const double v = M[(size_t)l * n + k];
          const float fv = (float)v;
          f32[(size_t)l * ld + k] = fv;
          const unsigned short h = host_f2bf(fv);
          hl[(size_t)l * ld + k] = h;
          hl[plane + (size_t)l * ld + k] = host_f2bf((float)(v - (double)host_bf2f(h)));
        }
      hipError_t e;
      if ((e = hipMalloc(&p->lp_f32[a][d], f32.size() * 4)) != hipSuccess ||
          (e = hipMemcpy(p->lp_f32[a][d], f32.data(), f32.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
          (e = hipMalloc(&p->lp_hi[a][d], hl.size() * 2)) != hipSuccess ||
          (e = hipMemcpy(p->lp_hi[a][d], hl.data(), hl.size() * 2, hipMemcpyHostToDevice)) != hipSuccess) {
        release_lowp(p);
        return hip_fail(e, "low-precision factor upload");
      }
      p->lp_lo[a][d] = (unsigned short*)p->lp_hi[a][d] + plane;
    }
  }
  p->lp_ready = 1;
  return SEM_OK;
}

// Workspace layout of the low-precision solves (see workspace_need).
sem_status lp_prepare(sem_plan* p, sem_prec prec, LpWork* w) {
  if (prec != SEM_F32 && prec != SEM_BF16 && prec != SEM_BF16X3) return set_error(SEM_EINVAL, "unknown precision");
  if (p->dims[0] > 46340 || (long)p->dims[1] * p->dims[2] > 0x7fffffffL ||
      (long)p->dims[0] * p->dims[2] > 0x7fffffffL || (long)p->dims[0] * p->dims[1] > 0x7fffffffL)
    return set_error(SEM_EINVAL, "problem too large for the low-precision kernels");
  sem_status st = ensure_lowp(p);
  if (st != SEM_OK) return st;
  void* ws = nullptr;
  st = plan_workspace(p, workspace_need(p, prec), &ws);
  if (st != SEM_OK) return st;
  char* b = (char*)ws;
  const bool split = lp_split(prec);
  const size_t rbytes = lp_r_bytes(p, prec);
  const size_t tbytes = ((lp_tmp_elems(p, prec) * lp_elem(prec) + 255) / 256) * 256;
  w->prec = prec;
  w->r = b;
  w->t0 = b + rbytes;
  w->t1 = b + rbytes + tbytes;
  w->norms = (unsigned long long*)(b + rbytes + 2 * tbytes);
  w->rkind = prec == SEM_F32 ? 1 : split ? 3 : 2;
  w->ldr = lp_pitch(p->dims[2], prec);
  w->rplane = split ? (long)lp_r_elems(p, prec) : 0;
  w->tplane = split ? (long)lp_tmp_elems(p, prec) : 0;
  return SEM_OK;
}

// One low-precision FD application  u (+)= S_3 [ (F_3 src) / (alpha + b1 L + b2 L^2) ].
//  f64_src != null: the FP64 right-hand side in the caller's layout (FP32 reads it
//    directly; the BF16 modes first convert it into w.r);
//  f64_src == null: src is w.r, written by the residual kernel in the
//    intermediate format (row pitch w.ldr).
//  first = 1 stores u = delta, else u += delta; norms (may be null) receive
//  max|delta| and max|u| as FP64 bit patterns (the caller zeroes them).
hipError_t lp_fd(sem_plan* p, const LpWork& w, const Spectral& sp, const double* f64_src, double* u, int first,
                 unsigned long long* norms) {
  const sem_prec prec = w.prec;
  const int nx = p->dims[0], ny = p->dims[1], nz = p->dims[2];
  const int mode = prec == SEM_F32 ? LP_F32 : prec == SEM_BF16 ? LP_BF16 : LP_BF16X3;
  const bool dma = mode != LP_F32;
  const int lpk = mode == LP_F32 ? 1 : 2;  // intermediate kind (FP32 / BF16 planes)
  if (f64_src && dma) {
    hipError_t e = launch_to_lowp(f64_src, w.r, w.rplane, mode == LP_BF16X3 ? 1 : 0, p->dims, w.ldr, p->stream);
    if (e != hipSuccess) return e;
  }
  const bool from_r = !f64_src || dma;
  const void* src = from_r ? w.r : (const void*)f64_src;
  void* t0 = w.t0;
  void* t1 = w.t1;
  const long tplane = w.tplane;
  // the six passes: (input, ldx, A, B, K) -> (output, ldy); axis contracted = K's axis
  struct Step {
    const void* x;
    int ldx, A, B, K, axis, dir;
    void* y;
    int ldy, in_kind, out_kind, epi;
    long xplane, yplane;
  };
  const int in0 = from_r ? lpk : 0;
  const int px = lp_pitch(nx, prec), py = lp_pitch(ny, prec), pz = lp_pitch(nz, prec);
  const Step st[6] = {
      {src, from_r ? w.ldr : nz, nx, ny, nz, 2, 0, t0, py, in0, lpk, EPI_STORE, w.rplane, tplane},
      {t0, py, nz, nx, ny, 1, 0, t1, px, lpk, lpk, EPI_STORE, tplane, tplane},
      {t1, px, ny, nz, nx, 0, 0, t0, pz, lpk, lpk, EPI_DIVIDE, tplane, tplane},
      {t0, pz, nx, ny, nz, 2, 1, t1, py, lpk, lpk, EPI_STORE, tplane, tplane},
      {t1, py, nz, nx, ny, 1, 1, t0, px, lpk, lpk, EPI_STORE, tplane, tplane},
      {t0, px, ny, nz, nx, 0, 1, u, nz, lpk, 0, EPI_ACCUM, tplane, 0},
  };
  for (int s = 0; s < 6; ++s) {
    LpPass ps;
    ps.mode = mode;
    ps.x = st[s].x;
    ps.ldx = st[s].ldx;
    ps.P = (long)st[s].A * st[s].B;
    ps.K = st[s].K;
    ps.y = st[s].y;
    ps.ldy = st[s].ldy;
    ps.A = st[s].A;
    ps.B = st[s].B;
    ps.L = st[s].K;
    const int axis = st[s].axis, dir = st[s].dir;
    ps.f_hi = mode == LP_F32 ? p->lp_f32[axis][dir] : p->lp_hi[axis][dir];
    ps.f_lo = mode == LP_F32 ? nullptr : p->lp_lo[axis][dir];
    ps.ldf = p->lp_ld[axis];
    ps.in_kind = st[s].in_kind;
    ps.out_kind = st[s].out_kind;
    ps.epi_kind = st[s].epi;
    if (mode == LP_BF16X3) {
      ps.xplane = st[s].xplane;
      ps.yplane = st[s].yplane;
      ps.fplane = (long)ps.ldf * ps.ldf;
    }
    if (st[s].epi == EPI_DIVIDE) {
      // output (x, y, z): l = x mode, a = y mode, b = z mode
      ps.epi.l0 = p->d_lam[0];
      ps.epi.l1 = p->d_lam[1];
      ps.epi.l2 = p->d_lam[2];
      ps.epi.alpha = sp.alpha;
      ps.epi.b1 = sp.b1;
      ps.epi.b2 = sp.b2;
    }
    if (st[s].epi == EPI_ACCUM) {
      ps.epi.first = first;
      ps.epi.norms = norms;
    }
    hipError_t e;
    if (dma) {
      if (!dma_supported(ps)) return hipErrorInvalidValue;
      e = launch_mode_dma(ps, p->stream);
    } else {
      e = launch_mode_lp(ps, p->stream);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// FP64 FD application u = S_3 [ (F_3 f) / (alpha + b1 L + b2 L^2) ]; tmp holds N
// doubles; u may alias f.
hipError_t fd64(sem_plan* p, const Spectral& sp, const double* f, double* u, double* tmp) {
  EpiArgs none;
  EpiArgs div;
  div.lx = p->d_lam[0];
  div.ly = p->d_lam[1];
  div.lz = p->d_lam[2];
  div.alpha = sp.alpha;
  div.b1 = sp.b1;
  div.b2 = sp.b2;
  div.kind = sp.kind;
  div.param = sp.param;
  div.nz = p->dims[2];
  hipError_t e;
  if ((e = launch_mode_f64(f, tmp, p->d_gf[2], p->ld[2], p->dims, 2, EPI_STORE, none, p->stream)) != hipSuccess ||
      (e = launch_mode_f64(tmp, u, p->d_gf[1], p->ld[1], p->dims, 1, EPI_STORE, none, p->stream)) != hipSuccess ||
      (e = launch_mode_f64(u, tmp, p->d_gf[0], p->ld[0], p->dims, 0, sp.kind ? EPI_SPECTRAL : EPI_DIVIDE, div,
                           p->stream)) != hipSuccess ||
      (e = launch_mode_f64(tmp, u, p->d_gb[2], p->ld[2], p->dims, 2, EPI_STORE, none, p->stream)) != hipSuccess ||
      (e = launch_mode_f64(u, tmp, p->d_gb[1], p->ld[1], p->dims, 1, EPI_STORE, none, p->stream)) != hipSuccess ||
      (e = launch_mode_f64(tmp, u, p->d_gb[0], p->ld[0], p->dims, 0, EPI_STORE, none, p->stream)) != hipSuccess)
    return e;
  return hipSuccess;
}

hipError_t zero_norms(unsigned long long* norms, hipStream_t stream) {
  zero_u64_kernel<<<1, 64, 0, stream>>>(norms, 2);
  return hipGetLastError();
}

}  // namespace semfd

using namespace semfd;

extern "C" sem_status sem_solve_refined(sem_plan* p, sem_prec prec, double tol, int max_iter, const double* f,
                                        double* u, int* iters, double* last_update_rel) {
  if (!p || !f || !u || max_iter < 1 || !(tol >= 0.0) || !std::isfinite(tol))
    return set_error(SEM_EINVAL, "sem_solve_refined: invalid argument");
  if (f == u) return set_error(SEM_EINVAL, "sem_solve_refined: u must not alias f");
  if (iters) *iters = 0;
  if (last_update_rel) *last_update_rel = NAN;
  if (prec == SEM_F64) {
    sem_status st = sem_solve(p, f, u);
    if (st == SEM_OK && iters) *iters = 1;
    if (st == SEM_OK && last_update_rel) *last_update_rel = 0.0;
    return st;
  }
  if (prec != SEM_F32 && prec != SEM_BF16 && prec != SEM_BF16X3)
    return set_error(SEM_EINVAL, "sem_solve_refined: unknown precision");
  LpWork w;
  sem_status st = lp_prepare(p, prec, &w);
  if (st != SEM_OK) return st;
  const double* hb[3] = {p->d_hb[0], p->d_hb[1], p->d_hb[2]};
  const Spectral sp{p->alpha, 1.0, 0.0};
  ResidualArgs ra;  // r = f - alpha u - H_3 u in the intermediate format
  ra.periodic = p->per_mask;
  ra.v = u;
  ra.f = f;
  ra.r = w.r;
  ra.r_kind = w.rkind;
  ra.ldr = w.ldr;
  ra.rplane = w.rplane;
  ra.cf = 1.0;
  ra.cd = p->alpha;
  ra.ch = 1.0;

  double prev = INFINITY, prev2 = INFINITY;
  for (int it = 0; it < max_iter; ++it) {
    hipError_t e;
    if (it > 0 && (e = launch_residual(ra, hb, p->k, p->dims, p->stream)) != hipSuccess)
      return hip_fail(e, "sem_solve_refined: residual");
    if ((e = zero_norms(w.norms, p->stream)) != hipSuccess) return hip_fail(e, "sem_solve_refined: norm reset");
    if ((e = lp_fd(p, w, sp, it == 0 ? f : nullptr, u, it == 0 ? 1 : 0, w.norms)) != hipSuccess)
      return hip_fail(e, "sem_solve_refined: low-precision solve");
    unsigned long long hn[2];
    if ((e = hipMemcpyAsync(hn, w.norms, sizeof(hn), hipMemcpyDeviceToHost, p->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(p->stream)) != hipSuccess)
      return hip_fail(e, "sem_solve_refined: norm readback");
    double dmax, umax;
    std::memcpy(&dmax, &hn[0], 8);
    std::memcpy(&umax, &hn[1], 8);
    if (iters) *iters = it + 1;
    if (!std::isfinite(dmax) || !std::isfinite(umax))
      return set_error(SEM_ENONFINITE, "sem_solve_refined: non-finite update");
    const double rel = umax > 0 ? dmax / umax : (dmax > 0 ? INFINITY : 0.0);
    if (last_update_rel) *last_update_rel = rel;
    if (refine_converged(rel, prev, prev2, tol)) return SEM_OK;
    if (it >= 2 && rel > prev && prev > prev2)
      return set_error(SEM_ENOCONV, "sem_solve_refined: updates grow; refinement diverges at this precision");
    prev2 = prev;
    prev = rel;
  }
  if (tol > 0) return set_error(SEM_ENOCONV, "sem_solve_refined: tolerance not met within max_iter");
  return SEM_OK;
}

extern "C" sem_status sem_solve_lowp(sem_plan* p, sem_prec prec, const double* f, double* u) {
  if (!p || !f || !u) return set_error(SEM_EINVAL, "sem_solve_lowp: null argument");
  if (f == u) return set_error(SEM_EINVAL, "sem_solve_lowp: u must not alias f");
  if (prec == SEM_F64) return sem_solve(p, f, u);
  if (prec != SEM_F32 && prec != SEM_BF16 && prec != SEM_BF16X3)
    return set_error(SEM_EINVAL, "sem_solve_lowp: unknown precision");
  LpWork w;
  sem_status st = lp_prepare(p, prec, &w);
  if (st != SEM_OK) return st;
  const hipError_t e = lp_fd(p, w, Spectral{p->alpha, 1.0, 0.0}, f, u, 1, nullptr);
  if (e != hipSuccess) return hip_fail(e, "sem_solve_lowp");
  return SEM_OK;
}
