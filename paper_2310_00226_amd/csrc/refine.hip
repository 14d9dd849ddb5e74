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
#include <cstdio>
#include <string>
#include <cstring>
#include <vector>

#include "kernels.h"
#include "plan_internal.h"
#include "tune.h"

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

inline int pad32(int n) { return (n + 31) / 32 * 32; }
// reflection split of axis a: representatives, antisymmetric modes, folded node
// row pitch (v+ then v-), split mode row pitch (symmetric block, antisymmetric
// block, each from a 32-element boundary)
inline int nrep_of(const sem_plan* p, int a) { return p->ax[a].nrep; }
inline int fold_pitch(const sem_plan* p, int a) { return 2 * pad32(p->ax[a].nrep); }
inline int mode_pitch(const sem_plan* p, int a) {
  return pad32(p->ax[a].nrep) + pad32(std::max(p->ax[a].nodd, 1));
}
// row pitch of the folded correction (FP32, z'' = 2 nrep_z values)
inline int dpitch(const sem_plan* p) { return pad8(2 * p->ax[2].nrep); }

// FP32: largest of the three rotated padded layouts (z,x,y'), (y,z,x'), (x,y,z').
// BF16 modes: largest of the reflection-split layouts of lp_fd (BF16 elements per
// plane; the FP32 correction of the last pass, 2 elements per value, included).
size_t lp_tmp_elems(const sem_plan* p, sem_prec prec) {
  const size_t nx = p->dims[0], ny = p->dims[1], nz = p->dims[2];
  if (prec == SEM_F32)
    return std::max({nz * nx * (size_t)lp_pitch((int)ny, prec), ny * nz * (size_t)lp_pitch((int)nx, prec),
                     nx * ny * (size_t)lp_pitch((int)nz, prec)});
  const size_t rx = 2 * (size_t)nrep_of(p, 0), ry = 2 * (size_t)nrep_of(p, 1), rz = 2 * (size_t)nrep_of(p, 2);
  const size_t corr = rx * ry * (size_t)dpitch(p) * 2 / (prec == SEM_BF16X3 ? 2 : 1);
  return std::max({nx * ny * (size_t)fold_pitch(p, 2), nz * nx * (size_t)fold_pitch(p, 1),
                   ny * nz * (size_t)fold_pitch(p, 0), nx * ny * (size_t)mode_pitch(p, 2),
                   rz * nx * (size_t)mode_pitch(p, 1), ry * rz * (size_t)mode_pitch(p, 0), corr});
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
      (void)hipFree(p->lpf[a][d]);
      p->lp_f32[a][d] = p->lp_hi[a][d] = p->lp_lo[a][d] = p->lpf[a][d] = nullptr;
    }
  for (int a = 0; a < 3; ++a) {
    (void)hipFree(p->d_lamf[a]);
    p->d_lamf[a] = nullptr;
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
    // reflection-split factors (BF16 hi / lo): forward [modes][representatives],
    // backward [representatives][modes of the block]
    const semfd::AxisData& ax = p->ax[a];
    const int nr = ax.nrep, no = ax.nodd, frow2 = pad256(nr), ldf = pad32(nr);
    const int rows_f = frow2 + pad256(std::max(no, 1)), rows_b = 2 * frow2;
    p->lpf_ld[a] = ldf;
    p->lpf_frow2[a] = frow2;
    p->lpf_plane[a] = (long)std::max(rows_f, rows_b) * ldf;
    for (int d = 0; d < 2; ++d) {
      const size_t pl = (size_t)p->lpf_plane[a];
      std::vector<unsigned short> hl(2 * pl, 0);
      auto put = [&](int row, int col, double v) {
        const float fv = (float)v;
        const unsigned short h = host_f2bf(fv);
        hl[(size_t)row * ldf + col] = h;
        hl[pl + (size_t)row * ldf + col] = host_f2bf((float)(v - (double)host_bf2f(h)));
      };
      if (d == 0) {
        for (int t = 0; t < n; ++t)
          for (int r = 0; r < nr; ++r) put(t < nr ? t : frow2 + (t - nr), r, ax.ffold[(size_t)t * nr + r]);
      } else {
        for (int r = 0; r < nr; ++r) {
          for (int t = 0; t < nr; ++t) put(r, t, ax.bfold_sym[(size_t)r * nr + t]);
          for (int t = 0; t < no; ++t) put(frow2 + r, t, ax.bfold_anti[(size_t)r * no + t]);
        }
      }
      hipError_t e;
      if ((e = hipMalloc(&p->lpf[a][d], hl.size() * 2)) != hipSuccess ||
          (e = hipMemcpy(p->lpf[a][d], hl.data(), hl.size() * 2, hipMemcpyHostToDevice)) != hipSuccess) {
        release_lowp(p);
        return hip_fail(e, "folded factor upload");
      }
    }
    hipError_t e;
    if ((e = hipMalloc(&p->d_lamf[a], sizeof(double) * n)) != hipSuccess ||
        (e = hipMemcpy(p->d_lamf[a], ax.lam_fold.data(), sizeof(double) * n, hipMemcpyHostToDevice)) != hipSuccess) {
      release_lowp(p);
      return hip_fail(e, "folded eigenvalue upload");
    }
  }
  p->lp_ready = 1;
  return SEM_OK;
}

// Workspace layout of the low-precision solves (see workspace_need) inside ws.
sem_status lp_layout(sem_plan* p, sem_prec prec, void* ws, LpWork* w) {
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

sem_status lp_check(const sem_plan* p, sem_prec prec) {
  if (prec != SEM_F32 && prec != SEM_BF16 && prec != SEM_BF16X3) return set_error(SEM_EINVAL, "unknown precision");
  if (p->dims[0] > 46340 || (long)p->dims[1] * p->dims[2] > 0x7fffffffL ||
      (long)p->dims[0] * p->dims[2] > 0x7fffffffL || (long)p->dims[0] * p->dims[1] > 0x7fffffffL)
    return set_error(SEM_EINVAL, "problem too large for the low-precision kernels");
  return SEM_OK;
}

// Low-precision factors and the plan workspace laid out for prec; with tune, the
// launch shapes of prec are tuned (once per plan, see lp_tune).
sem_status lp_prepare(sem_plan* p, sem_prec prec, LpWork* w, bool tune) {
  sem_status st = lp_check(p, prec);
  if (st != SEM_OK) return st;
  st = ensure_lowp(p);
  if (st != SEM_OK) return st;
  void* ws = nullptr;
  st = plan_workspace(p, workspace_need(p, prec), &ws);
  if (st != SEM_OK) return st;
  st = lp_layout(p, prec, ws, w);
  if (st != SEM_OK || !tune) return st;
  return lp_tune(p, *w);
}

// Low-precision factors only (the caller provides the workspace, lp_layout).
sem_status lp_factors(sem_plan* p, sem_prec prec) {
  sem_status st = lp_check(p, prec);
  if (st != SEM_OK) return st;
  return ensure_lowp(p);
}

// BF16 / split-BF16 FD application on the reflection-split transforms:
//   fold z -> (z fwd, fold y) -> (y fwd, fold x) -> (x fwd, divide) -> z bwd -> y bwd
//   -> x bwd -> unfold + accumulate.
// Each forward pass contracts the folded node axis blockwise (symmetric modes with
// v+, antisymmetric with v-) and writes its output rows in folded mode order; the
// first two also fold the axis the next pass contracts.  Each backward pass
// contracts a mode axis blockwise and writes the folded node form e_r, o_r of its
// axis (rows), which only the final kernel resolves into nodes (u_r = e_r + o_r,
// u_R(r) = e_r - o_r on every axis) while adding the correction to u.
static void fold_axes(const sem_plan* p, FoldAxis fa[3]) {
  for (int a = 0; a < 3; ++a) {
    fa[a].nrep = p->ax[a].nrep;
    fa[a].pad = pad32(p->ax[a].nrep);
    fa[a].per = p->bc[a] == SEM_BC_PERIODIC ? 1 : 0;
  }
}

void lp_fold_axes(const sem_plan* p, FoldAxis fa[3]) { fold_axes(p, fa); }
int lp_fold_pitch_z(const sem_plan* p) { return fold_pitch(p, 2); }

// Pass s (0..5) of the reflection-split sequence: t1 -> t0 -> t1 -> t0 -> t1 -> t0 -> t1.
static LpPass folded_pass(sem_plan* p, const LpWork& w, const Spectral& sp, int s) {
  const int nx = p->dims[0], ny = p->dims[1], nz = p->dims[2];
  const int ry = p->ax[1].nrep, rz = p->ax[2].nrep;
  struct Step {
    int ldx, A, B, axis, dir, ldy, out_kind, epi, col, baxis;
  };
  // forward: K = representatives of the contracted axis (both blocks), rows =
  // n modes (nrep symmetric, nodd antisymmetric); backward: K = modes of the block,
  // rows = 2 nrep (e then o)
  const Step st[6] = {
      {fold_pitch(p, 2), nx, ny, 2, 0, fold_pitch(p, 1), 2, EPI_STORE, COL_FOLD, 1},
      {fold_pitch(p, 1), nz, nx, 1, 0, fold_pitch(p, 0), 2, EPI_STORE, COL_FOLD, 0},
      {fold_pitch(p, 0), ny, nz, 0, 0, mode_pitch(p, 2), 2, EPI_DIVIDE, COL_SPLIT, 2},
      {mode_pitch(p, 2), nx, ny, 2, 1, mode_pitch(p, 1), 2, EPI_STORE, COL_SPLIT, 1},
      {mode_pitch(p, 1), 2 * rz, nx, 1, 1, mode_pitch(p, 0), 2, EPI_STORE, COL_SPLIT, 0},
      {mode_pitch(p, 0), 2 * ry, 2 * rz, 0, 1, dpitch(p), 1, EPI_STORE, COL_PLAIN, 2},
  };
  const Step& q = st[s];
  const int a = q.axis;
  const semfd::AxisData& ax = p->ax[a];
  LpPass ps;
  ps.mode = w.prec == SEM_BF16 ? LP_BF16 : LP_BF16X3;
  ps.x = (s % 2 == 0) ? w.t1 : w.t0;
  ps.y = (s % 2 == 0) ? w.t0 : w.t1;
  ps.ldx = q.ldx;
  ps.A = q.A;
  ps.B = q.B;
  ps.P = (long)q.A * q.B;
  ps.ldy = q.ldy;
  ps.f_hi = p->lpf[a][q.dir];
  ps.ldf = p->lpf_ld[a];
  ps.fplane = p->lpf_plane[a];
  ps.in_kind = 2;
  ps.out_kind = q.out_kind;
  ps.epi_kind = q.epi;
  ps.xplane = w.tplane;
  ps.yplane = q.out_kind == 2 ? w.tplane : 0;
  ps.frow2 = p->lpf_frow2[a];
  ps.koff2 = pad32(ax.nrep);
  if (q.dir == 0) {  // forward: blocks of nrep and nodd modes over the representatives
    ps.K = ax.nrep;
    ps.L = ax.nrep;
    ps.K2 = ax.nodd > 0 ? ax.nrep : 0;
    ps.L2 = ax.nodd;
  } else {  // backward: e rows over the symmetric modes, o rows over the antisymmetric
    ps.K = ax.nrep;
    ps.L = ax.nrep;
    ps.K2 = std::max(ax.nodd, 1);  // nodd = 0: one zero chunk, o rows = 0
    ps.L2 = ax.nrep;
  }
  ps.col = q.col;
  if (q.col == COL_FOLD || q.col == COL_SPLIT) {
    const int bx = q.baxis;
    ps.bsym = p->ax[bx].nrep;
    ps.bpad = pad32(p->ax[bx].nrep);
    ps.bn = p->dims[bx];
    ps.bper = p->bc[bx] == SEM_BC_PERIODIC ? 1 : 0;
  }
  if (q.epi == EPI_DIVIDE) {
    // output (x modes, y modes, z modes), all in folded mode order
    ps.epi.l0 = p->d_lamf[0];
    ps.epi.l1 = p->d_lamf[1];
    ps.epi.l2 = p->d_lamf[2];
    ps.epi.alpha = sp.alpha;
    ps.epi.b1 = sp.b1;
    ps.epi.b2 = sp.b2;
  }
  if (p->tuned[w.prec]) ps.tile_group = p->tune_choice[w.prec][s];
  return ps;
}

static hipError_t lp_fd_folded(sem_plan* p, const LpWork& w, const Spectral& sp, const double* f64_src, double* u,
                               int first, unsigned long long* norms) {
  const int split = w.prec == SEM_BF16X3 ? 1 : 0;
  FoldAxis fa[3];
  fold_axes(p, fa);
  hipError_t e;
  // folded right-hand side into t1
  if (w.input_in_t1)
    e = hipSuccess;
  else if (f64_src)
    e = launch_to_lowp(f64_src, w.t1, w.tplane, split, p->dims, fold_pitch(p, 2), &fa[2], p->stream);
  else
    e = launch_fold_lowp(w.r, w.rplane, w.ldr, w.t1, w.tplane, fold_pitch(p, 2), split, p->dims, fa[2], p->stream);
  if (e != hipSuccess) return e;
  for (int s = 0; s < 6; ++s) {
    const LpPass ps = folded_pass(p, w, sp, s);
    if (!dma_supported(ps)) return hipErrorInvalidValue;
    if ((e = launch_mode_dma(ps, p->stream)) != hipSuccess) return e;
  }
  return launch_unfold_accum((const float*)w.t1, dpitch(p), u, p->dims, fa, first, norms, p->stream, w.unfold_dot);
}

// Pass s (0..5) of the FP32 sequence  src -> t0 -> t1 -> t0 -> t1 -> t0 -> u.
// With u == nullptr the last pass stores FP32 into t1 instead of accumulating
// into u (the stand-in the tuner times).
static LpPass f32_pass(sem_plan* p, const LpWork& w, const Spectral& sp, int s, const double* f64_src, double* u,
                       int first, unsigned long long* norms) {
  const int nx = p->dims[0], ny = p->dims[1], nz = p->dims[2];
  const sem_prec prec = SEM_F32;
  const bool from_r = !f64_src;
  const void* src = from_r ? w.r : (const void*)f64_src;
  const int px = lp_pitch(nx, prec), py = lp_pitch(ny, prec), pz = lp_pitch(nz, prec);
  struct Step {
    const void* x;
    int ldx, A, B, K, axis, dir;
    void* y;
    int ldy, in_kind, out_kind, epi;
  };
  const int in0 = from_r ? 1 : 0;
  const Step st[6] = {
      {src, from_r ? w.ldr : nz, nx, ny, nz, 2, 0, w.t0, py, in0, 1, EPI_STORE},
      {w.t0, py, nz, nx, ny, 1, 0, w.t1, px, 1, 1, EPI_STORE},
      {w.t1, px, ny, nz, nx, 0, 0, w.t0, pz, 1, 1, EPI_DIVIDE},
      {w.t0, pz, nx, ny, nz, 2, 1, w.t1, py, 1, 1, EPI_STORE},
      {w.t1, py, nz, nx, ny, 1, 1, w.t0, px, 1, 1, EPI_STORE},
      {w.t0, px, ny, nz, nx, 0, 1, u, nz, 1, 0, EPI_ACCUM},
  };
  const Step& q = st[s];
  LpPass ps;
  ps.mode = LP_F32;
  ps.x = q.x;
  ps.ldx = q.ldx;
  ps.P = (long)q.A * q.B;
  ps.K = q.K;
  ps.y = q.y;
  ps.ldy = q.ldy;
  ps.A = q.A;
  ps.B = q.B;
  ps.L = q.K;
  ps.f_hi = p->lp_f32[q.axis][q.dir];
  ps.ldf = p->lp_ld[q.axis];
  ps.in_kind = q.in_kind;
  ps.out_kind = q.out_kind;
  ps.epi_kind = q.epi;
  if (q.epi == EPI_DIVIDE) {
    // output (x, y, z): l = x mode, a = y mode, b = z mode
    ps.epi.l0 = p->d_lam[0];
    ps.epi.l1 = p->d_lam[1];
    ps.epi.l2 = p->d_lam[2];
    ps.epi.alpha = sp.alpha;
    ps.epi.b1 = sp.b1;
    ps.epi.b2 = sp.b2;
  }
  if (q.epi == EPI_ACCUM) {
    if (u) {
      ps.epi.first = first;
      ps.epi.norms = norms;
    } else {  // tuner stand-in: FP32 store of the same shape into t1 (pass 3's layout)
      ps.y = w.t1;
      ps.ldy = pz;
      ps.out_kind = 1;
      ps.epi_kind = EPI_STORE;
    }
  }
  if (p->tuned[SEM_F32]) ps.tile_rows = p->tune_choice[SEM_F32][s];
  return ps;
}

// One low-precision FD application  u (+)= S_3 [ (F_3 src) / (alpha + b1 L + b2 L^2) ].
//  f64_src != null: the FP64 right-hand side in the caller's layout (FP32 reads it
//    directly; the BF16 modes fold and convert it first);
//  f64_src == null: src is w.r, written by the residual kernel in the
//    intermediate format (row pitch w.ldr).
//  first = 1 stores u = delta, else u += delta; norms (may be null) receive
//  max|delta| and max|u| as FP64 bit patterns (the caller zeroes them).
hipError_t lp_fd(sem_plan* p, const LpWork& w, const Spectral& sp, const double* f64_src, double* u, int first,
                 unsigned long long* norms) {
  if (w.prec != SEM_F32) return lp_fd_folded(p, w, sp, f64_src, u, first, norms);
  for (int s = 0; s < 6; ++s) {
    const hipError_t e = launch_mode_lp(f32_pass(p, w, sp, s, f64_src, u, first, norms), p->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---- autotuning of the launch shapes -------------------------------------------
// FP32 passes: factor-tile rows 128, 96, 64 or 32; BF16 passes: tile order group
// of 1 or 4 p-strips, with one block per tile or one block per CU looping over
// the tiles (DMA_PERSIST + group).  Each pass geometry is timed once (one warm-up launch, the
// fastest of three), on the plan's own workspace, and the choice is kept in the
// plan and in the tuning cache (key: architecture, kernel, output layout, and
// log2 buckets of rows, contraction length and tensor rows), so plans of similar
// size skip the timing, also in later processes with SEM_TUNE_CACHE.
static const char* arch_name(const sem_plan* p) {
  static thread_local char name[64];
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, p->device) != hipSuccess) return "unknown";
  std::snprintf(name, sizeof(name), "%s", prop.gcnArchName);
  for (char* c = name; *c; ++c)
    if (*c == ':') *c = '_';
  return name;
}

static std::string pass_key(const sem_plan* p, const LpPass& ps) {
  char buf[192];
  std::snprintf(buf, sizeof(buf), "%s|%s|epi%d|col%d|out%d|L%d|K%d|P%d", arch_name(p),
                ps.mode == LP_F32 ? "f32" : ps.mode == LP_BF16 ? "bf16" : "bf16x3", ps.epi_kind, ps.col,
                ps.out_kind, tune_bucket(ps.L + ps.L2), tune_bucket(ps.K), tune_bucket(ps.P));
  return buf;
}

static hipError_t time_pass(sem_plan* p, const LpPass& ps, float* best_ms) {
  hipEvent_t t0, t1;
  hipError_t e;
  if ((e = hipEventCreate(&t0)) != hipSuccess) return e;
  if ((e = hipEventCreate(&t1)) != hipSuccess) {
    (void)hipEventDestroy(t0);
    return e;
  }
  auto launch = [&]() { return ps.mode == LP_F32 ? launch_mode_lp(ps, p->stream) : launch_mode_dma(ps, p->stream); };
  float best = INFINITY;
  e = launch();  // warm-up
  for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
    float ms = 0.f;
    if ((e = hipEventRecord(t0, p->stream)) == hipSuccess && (e = launch()) == hipSuccess &&
        (e = hipEventRecord(t1, p->stream)) == hipSuccess && (e = hipEventSynchronize(t1)) == hipSuccess &&
        (e = hipEventElapsedTime(&ms, t0, t1)) == hipSuccess)
      best = std::min(best, ms);
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  *best_ms = best;
  return e;
}

sem_status lp_tune(sem_plan* p, const LpWork& w) {
  const sem_prec prec = w.prec;
  if (p->tuned[prec]) return SEM_OK;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(p->stream, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone)
    return SEM_OK;  // no timing under capture: the rule-based shapes stay
  const Spectral sp{p->alpha, 1.0, 0.0};
  static const int rows_cand[4] = {128, 96, 64, 32};
  static const int group_cand[4] = {1, 4, DMA_PERSIST + 1, DMA_PERSIST + 4};
  for (int s = 0; s < 6; ++s) {
    LpPass ps = prec == SEM_F32 ? f32_pass(p, w, sp, s, nullptr, nullptr, 1, nullptr) : folded_pass(p, w, sp, s);
    if (prec == SEM_F32) ps.in_kind = 1;  // first pass: time the FP32-input variant
    if (prec == SEM_F32 && s == 0) {
      ps.x = w.r;
      ps.ldx = w.ldr;
    }
    const std::string key = pass_key(p, ps);
    int choice = 0;
    if (!tune_lookup(key, &choice)) {
      const int* cand = prec == SEM_F32 ? rows_cand : group_cand;
      const int nc = 4;
      float best = INFINITY;
      for (int c = 0; c < nc; ++c) {
        if (prec == SEM_F32)
          ps.tile_rows = cand[c];
        else
          ps.tile_group = cand[c];
        float ms = INFINITY;
        const hipError_t e = time_pass(p, ps, &ms);
        if (e != hipSuccess) return hip_fail(e, "autotune");
        if (ms < best) {
          best = ms;
          choice = cand[c];
        }
      }
      tune_store(key, choice);
    }
    p->tune_choice[prec][s] = choice;
  }
  p->tuned[prec] = 1;
  return SEM_OK;
}

// FP64 FD application on the reflection-split transforms (the plan's folded
// blocks), two launches per mode product.  The antisymmetric blocks use only the
// nodd representatives that are not their own reflection (r = j + off, off = 1
// on periodic axes, whose node 0 is fixed; the fixed node of an odd
// non-periodic axis is the last representative), whose v- is not identically 0:
//  - z forward: the blocks read the unfolded z rows as v+ = x_r + x_R(r) or
//    v- = x_r - x_R(r) in their loads;
//  - y and x forward: a compact fold pass ([v+ of the nrep representatives |
//    v- of the nodd others], n rows) feeds plain block products;
//  - the forward blocks write the modes in folded order ([symmetric |
//    antisymmetric]), so the x product's multiplier reads the folded eigenvalues;
//  - backward (x, y, z): the symmetric block stores e_r at node r, the
//    antisymmetric block reads it back and stores u_r = e_r + o_r and
//    u_R(r) = e_r - o_r (at a fixed node e_r stays).
// Buffers: f -> tmp -> u -> tmp -> u -> tmp -> u -> tmp -> u (tmp: N doubles; u
// may alias f, which the first product alone reads).
hipError_t fd64(sem_plan* p, const Spectral& sp, const double* f, double* u, double* tmp) {
  const int nx = p->dims[0], ny = p->dims[1], nz = p->dims[2];
  const int r[3] = {p->ax[0].nrep, p->ax[1].nrep, p->ax[2].nrep};
  const int o[3] = {p->ax[0].nodd, p->ax[1].nodd, p->ax[2].nodd};
  const int n[3] = {nx, ny, nz};
  int per[3], off[3];
  for (int a = 0; a < 3; ++a) {
    per[a] = p->bc[a] == SEM_BC_PERIODIC ? 1 : 0;
    off[a] = per[a];
  }
  const long PZ = (long)nx * ny, QY = nz, PY = nx, QX = (long)ny * nz;
  EpiArgs none;
  EpiArgs plus_z, minus_z, unfold[3];
  plus_z.fold = 1;
  minus_z.fold = 2;
  plus_z.rn = minus_z.rn = nz;
  plus_z.rper = minus_z.rper = per[2];
  minus_z.roff = off[2];
  for (int a = 0; a < 3; ++a) {
    unfold[a].rn = n[a];
    unfold[a].rper = per[a];
    unfold[a].roff = off[a];
  }
  EpiArgs mul;
  mul.lx = p->d_lamf64[0];
  mul.ly = p->d_lamf64[1];
  mul.lz = p->d_lamf64[2];
  mul.alpha = sp.alpha;
  mul.b1 = sp.b1;
  mul.b2 = sp.b2;
  mul.kind = sp.kind;
  mul.param = sp.param;
  mul.nz = nz;
  EpiArgs mul_anti = mul;
  mul_anti.lx = p->d_lamf64[0] + r[0];
  const int epi = sp.kind ? EPI_SPECTRAL : EPI_DIVIDE;
  // antisymmetric blocks: forward factors start at row off (representative
  // off), backward factors at column off
  const double* gfa[3];
  const double* gba[3];
  for (int a = 0; a < 3; ++a) {
    gfa[a] = p->d_gff[a][1] + (size_t)off[a] * p->fld[a];
    gba[a] = p->d_gbf[a][1] + off[a];
  }
  hipStream_t s = p->stream;
  hipError_t e;
#define SEMFD_TRY(x) \
  if ((e = (x)) != hipSuccess) return e
  // z forward (NT shape, rows (x, y)), folding in the loads: f -> tmp (z modes)
  SEMFD_TRY(launch_mode_f64_part(f, tmp, p->d_gff[2][0], p->fld[2], PZ, r[2], r[2], 1, nz, nz, EPI_STORE, plus_z, s));
  SEMFD_TRY(launch_mode_f64_part(f, tmp + r[2], gfa[2], p->fld[2], PZ, o[2], o[2], 1, nz, nz, EPI_STORE, minus_z, s));
  // y: fold tmp -> u, forward (batched over x, inner z modes) u -> tmp
  SEMFD_TRY(launch_fold_f64(tmp, u, PY, ny, QY, r[1], per[1], s));
  SEMFD_TRY(launch_mode_f64_part(u, tmp, p->d_gff[1][0], p->fld[1], PY, r[1], r[1], QY, ny, ny, EPI_STORE, none, s));
  SEMFD_TRY(launch_mode_f64_part(u + (size_t)r[1] * QY, tmp + (size_t)r[1] * QY, gfa[1], p->fld[1], PY, o[1], o[1], QY,
                                 ny, ny, EPI_STORE, none, s));
  // x: fold tmp -> u, forward with the multiplier u -> tmp
  SEMFD_TRY(launch_fold_f64(tmp, u, 1, nx, QX, r[0], per[0], s));
  SEMFD_TRY(launch_mode_f64_part(u, tmp, p->d_gff[0][0], p->fld[0], 1, r[0], r[0], QX, nx, nx, epi, mul, s));
  SEMFD_TRY(launch_mode_f64_part(u + (size_t)r[0] * QX, tmp + (size_t)r[0] * QX, gfa[0], p->fld[0], 1, o[0], o[0], QX,
                                 nx, nx, epi, mul_anti, s));
  // x backward: tmp (x modes) -> u (x nodes)
  SEMFD_TRY(launch_mode_f64_part(tmp, u, p->d_gbf[0][0], p->fld[0], 1, r[0], r[0], QX, nx, nx, EPI_STORE, none, s));
  SEMFD_TRY(launch_mode_f64_part(tmp + (size_t)r[0] * QX, u, gba[0], p->fld[0], 1, o[0], o[0], QX, nx, nx, EPI_UNFOLD,
                                 unfold[0], s));
  // y backward: u -> tmp
  SEMFD_TRY(launch_mode_f64_part(u, tmp, p->d_gbf[1][0], p->fld[1], PY, r[1], r[1], QY, ny, ny, EPI_STORE, none, s));
  SEMFD_TRY(launch_mode_f64_part(u + (size_t)r[1] * QY, tmp, gba[1], p->fld[1], PY, o[1], o[1], QY, ny, ny, EPI_UNFOLD,
                                 unfold[1], s));
  // z backward: tmp -> u
  SEMFD_TRY(launch_mode_f64_part(tmp, u, p->d_gbf[2][0], p->fld[2], PZ, r[2], r[2], 1, nz, nz, EPI_STORE, none, s));
  SEMFD_TRY(launch_mode_f64_part(tmp + r[2], u, gba[2], p->fld[2], PZ, o[2], o[2], 1, nz, nz, EPI_UNFOLD, unfold[2], s));
#undef SEMFD_TRY
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

extern "C" sem_status sem_plan_tune(sem_plan* p, sem_prec prec) {
  if (!p) return set_error(SEM_EINVAL, "sem_plan_tune: null plan");
  if (prec != SEM_F32 && prec != SEM_BF16 && prec != SEM_BF16X3)
    return set_error(SEM_EINVAL, "sem_plan_tune: only SEM_F32, SEM_BF16 and SEM_BF16X3 have tunable shapes");
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(p->stream, &cap);
  if (e != hipSuccess) return hip_fail(e, "sem_plan_tune: stream");
  if (cap != hipStreamCaptureStatusNone) return set_error(SEM_EINVAL, "sem_plan_tune: the plan stream is capturing");
  p->tuned[prec] = 0;
  LpWork w;
  sem_status st = lp_prepare(p, prec, &w, true);
  if (st != SEM_OK) return st;
  if ((e = hipStreamSynchronize(p->stream)) != hipSuccess) return hip_fail(e, "sem_plan_tune");
  return SEM_OK;
}

extern "C" sem_status sem_plan_tuning(const sem_plan* p, sem_prec prec, int* tuned, int choice[6]) {
  if (!p || !tuned || !choice) return set_error(SEM_EINVAL, "sem_plan_tuning: null argument");
  if (prec != SEM_F32 && prec != SEM_BF16 && prec != SEM_BF16X3)
    return set_error(SEM_EINVAL, "sem_plan_tuning: only SEM_F32, SEM_BF16 and SEM_BF16X3 have tunable shapes");
  *tuned = p->tuned[prec];
  for (int s = 0; s < 6; ++s) choice[s] = p->tuned[prec] ? p->tune_choice[prec][s] : 0;
  return SEM_OK;
}

extern "C" sem_status sem_plan_set_tuning(sem_plan* p, sem_prec prec, const int choice[6]) {
  if (!p || !choice) return set_error(SEM_EINVAL, "sem_plan_set_tuning: null argument");
  if (prec != SEM_F32 && prec != SEM_BF16 && prec != SEM_BF16X3)
    return set_error(SEM_EINVAL, "sem_plan_set_tuning: only SEM_F32, SEM_BF16 and SEM_BF16X3 have tunable shapes");
  for (int s = 0; s < 6; ++s) {
    const int c = choice[s];
    const int g = c > DMA_PERSIST ? c - DMA_PERSIST : c;
    const bool ok = prec == SEM_F32 ? (c == 128 || c == 96 || c == 64 || c == 32) : (g == 1 || g == 2 || g == 4);
    if (!ok)
      return set_error(SEM_EINVAL, prec == SEM_F32 ? "sem_plan_set_tuning: FP32 tile rows must be 128, 96, 64 or 32"
                                                   : "sem_plan_set_tuning: BF16 shapes must be 1, 2, 4 or 17, 18, 20");
  }
  for (int s = 0; s < 6; ++s) p->tune_choice[prec][s] = choice[s];
  p->tuned[prec] = 1;
  return SEM_OK;
}

extern "C" sem_status sem_tune_stats(int* hits, int* misses, int* entries) {
  if (!hits || !misses || !entries) return set_error(SEM_EINVAL, "sem_tune_stats: null argument");
  tune_counts(hits, misses);
  *entries = tune_size();
  return SEM_OK;
}

extern "C" sem_status sem_lowp_pass(sem_plan* p, sem_prec prec, int pass, int reps) {
  if (!p) return set_error(SEM_EINVAL, "sem_lowp_pass: null plan");
  if (prec != SEM_F32 && prec != SEM_BF16 && prec != SEM_BF16X3)
    return set_error(SEM_EINVAL, "sem_lowp_pass: only SEM_F32, SEM_BF16 and SEM_BF16X3 run low-precision passes");
  if (pass < 0 || pass > 5 || reps < 1) return set_error(SEM_EINVAL, "sem_lowp_pass: pass in 0..5, reps >= 1");
  LpWork w;
  sem_status st = lp_prepare(p, prec, &w, true);
  if (st != SEM_OK) return st;
  const Spectral sp{p->alpha, 1.0, 0.0};
  const LpPass ps = prec == SEM_F32 ? f32_pass(p, w, sp, pass, nullptr, nullptr, 1, nullptr) : folded_pass(p, w, sp, pass);
  LpPass q = ps;
  if (prec == SEM_F32) {  // FP32 input throughout, the first pass from the residual buffer
    q.in_kind = 1;
    if (pass == 0) {
      q.x = w.r;
      q.ldx = w.ldr;
    }
  } else if (!dma_supported(q)) {
    return set_error(SEM_EINVAL, "sem_lowp_pass: pass geometry not supported");
  }
  for (int r = 0; r < reps; ++r) {
    const hipError_t e = prec == SEM_F32 ? launch_mode_lp(q, p->stream) : launch_mode_dma(q, p->stream);
    if (e != hipSuccess) return hip_fail(e, "sem_lowp_pass");
  }
  return SEM_OK;
}
