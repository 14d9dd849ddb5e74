// C ABI of the fast-diagonalisation solver (declarations and contracts: include/sem.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/sem.h"
#include "kernels.h"
#include "plan_host.h"
#include "plan_internal.h"

using namespace semfd;

namespace {

thread_local std::string g_last_error;

sem_status fail(sem_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

int host_threads() {
  unsigned hc = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(hc, 16u));
}

}  // namespace

namespace semfd {

sem_status hip_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) return fail(SEM_ENOMEM, "%s: %s", what, hipGetErrorString(e));
  return fail(SEM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

sem_status set_error(sem_status st, const char* msg) { return fail(st, "%s", msg); }

// Device copy of one factor in the G[m][l] = A[l][m] layout, zero-padded to ld x ld.
static hipError_t upload_factor(const std::vector<double>& A, int n, int ld, double** dst) {
  std::vector<double> g((size_t)ld * ld, 0.0);
  for (int l = 0; l < n; ++l)
    for (int m = 0; m < n; ++m) g[(size_t)m * ld + l] = A[(size_t)l * n + m];
  hipError_t e = hipMalloc(dst, sizeof(double) * g.size());
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, g.data(), sizeof(double) * g.size(), hipMemcpyHostToDevice);
}

static hipError_t upload_vec(const std::vector<double>& v, double** dst) {
  hipError_t e = hipMalloc(dst, sizeof(double) * std::max<size_t>(v.size(), 1));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, v.data(), sizeof(double) * v.size(), hipMemcpyHostToDevice);
}

// Reflection-split FP64 factors of axis a in the G[m][l] = A[l][m] layout of the
// FP64 kernels, fld columns (nrep rounded up to 128) and fld + 128 zero-padded
// rows, so that a block read at a row or column offset of one (the antisymmetric
// blocks skip the representatives that are their own reflection) keeps whole
// tiles inside: forward blocks A = (symmetric or antisymmetric modes) x
// representatives, backward blocks A = representatives x (modes of the block);
// and the folded eigenvalues.
static hipError_t upload_fold_factors(sem_plan* p, int a) {
  const semfd::AxisData& ax = p->ax[a];
  const int nr = ax.nrep, no = ax.nodd, ld = ((nr + 127) / 128) * 128;
  p->fld[a] = ld;
  std::vector<double> g[4];
  for (auto& v : g) v.assign((size_t)(ld + 128) * ld, 0.0);
  for (int l = 0; l < nr; ++l)
    for (int m = 0; m < nr; ++m) g[0][(size_t)m * ld + l] = ax.ffold[(size_t)l * nr + m];
  for (int j = 0; j < no; ++j)
    for (int m = 0; m < nr; ++m) g[1][(size_t)m * ld + j] = ax.ffold[(size_t)(nr + j) * nr + m];
  for (int r = 0; r < nr; ++r)
    for (int m = 0; m < nr; ++m) g[2][(size_t)m * ld + r] = ax.bfold_sym[(size_t)r * nr + m];
  for (int r = 0; r < nr; ++r)
    for (int m = 0; m < no; ++m) g[3][(size_t)m * ld + r] = ax.bfold_anti[(size_t)r * no + m];
  double** dst[4] = {&p->d_gff[a][0], &p->d_gff[a][1], &p->d_gbf[a][0], &p->d_gbf[a][1]};
  for (int i = 0; i < 4; ++i) {
    hipError_t e = hipMalloc(dst[i], sizeof(double) * g[i].size());
    if (e != hipSuccess) {
      *dst[i] = nullptr;
      return e;
    }
    if ((e = hipMemcpy(*dst[i], g[i].data(), sizeof(double) * g[i].size(), hipMemcpyHostToDevice)) != hipSuccess)
      return e;
  }
  return upload_vec(ax.lam_fold, &p->d_lamf64[a]);
}

sem_status plan_workspace(sem_plan* p, size_t need, void** out) {
  if (p->ws && p->ws_bytes >= need) {
    *out = p->ws;
    return SEM_OK;
  }
  if (p->ws_owned && p->ws) {
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "workspace resize");
    (void)hipFree(p->ws);
  }
  p->ws = nullptr;
  p->ws_bytes = 0;
  p->ws_owned = false;
  hipError_t e = hipMalloc(&p->ws, need);
  if (e != hipSuccess) {
    p->ws = nullptr;
    return hip_fail(e, "workspace allocation");
  }
  p->ws_bytes = need;
  p->ws_owned = true;
  *out = p->ws;
  return SEM_OK;
}

}  // namespace semfd

namespace {
bool valid_bc(sem_bc bc) { return bc == SEM_BC_DIRICHLET || bc == SEM_BC_NEUMANN || bc == SEM_BC_PERIODIC; }
// unknowns on an axis of ne elements: interior nodes (Dirichlet), all ne k + 1
// nodes (Neumann), or ne k with the node at b identified with the node at a
long axis_unknowns(sem_bc bc, long ne, long k) {
  return bc == SEM_BC_DIRICHLET ? ne * k - 1 : bc == SEM_BC_PERIODIC ? ne * k : ne * k + 1;
}
AxisSpec axis_spec(int k, int ne, double a, double b, sem_bc bc) {
  AxisSpec s{k, ne, a, b, bc == SEM_BC_DIRICHLET};
  s.periodic = bc == SEM_BC_PERIODIC;
  return s;
}
}  // namespace

extern "C" {

const char* sem_last_error(void) { return g_last_error.c_str(); }


sem_status sem_axis_host(int k, int ne, double a, double b, sem_bc bc, int* n, double* x, double* mass, double* lam,
                         double* S, double* F) {
  if (k < 1 || ne < 1 || !(a < b) || !std::isfinite(a) || !std::isfinite(b) || !valid_bc(bc))
    return fail(SEM_EINVAL, "sem_axis_host: invalid argument");
  if (bc == SEM_BC_DIRICHLET && ne * k < 2) return fail(SEM_EINVAL, "Dirichlet needs ne*k >= 2");
  const int nn = (int)axis_unknowns(bc, ne, k);
  if (n) *n = nn;
  if (!x && !mass && !lam && !S && !F) return SEM_OK;
  try {
    AxisData d;
    build_axis(axis_spec(k, ne, a, b, bc), d, host_threads());
    if (x) std::memcpy(x, d.x.data(), sizeof(double) * nn);
    if (mass) std::memcpy(mass, d.mass.data(), sizeof(double) * nn);
    if (lam) std::memcpy(lam, d.lam.data(), sizeof(double) * nn);
    if (S) std::memcpy(S, d.S.data(), sizeof(double) * nn * nn);
    if (F) std::memcpy(F, d.F.data(), sizeof(double) * nn * nn);
  } catch (const std::exception& ex) {
    return fail(SEM_EINVAL, "sem_axis_host: %s", ex.what());
  }
  return SEM_OK;
}

sem_status sem_axis_fold_host(int k, int ne, double a, double b, sem_bc bc, int* nrep, int* nodd, double* lam_fold,
                              double* ffold, double* bfold_sym, double* bfold_anti) {
  if (k < 1 || ne < 1 || !(a < b) || !std::isfinite(a) || !std::isfinite(b) || !valid_bc(bc))
    return fail(SEM_EINVAL, "sem_axis_fold_host: invalid argument");
  if (bc == SEM_BC_DIRICHLET && ne * k < 2) return fail(SEM_EINVAL, "Dirichlet needs ne*k >= 2");
  try {
    AxisData d;
    build_axis(axis_spec(k, ne, a, b, bc), d, host_threads());
    if (nrep) *nrep = d.nrep;
    if (nodd) *nodd = d.nodd;
    const size_t n = d.n, nr = d.nrep, no = d.nodd;
    if (lam_fold) std::memcpy(lam_fold, d.lam_fold.data(), sizeof(double) * n);
    if (ffold) std::memcpy(ffold, d.ffold.data(), sizeof(double) * n * nr);
    if (bfold_sym) std::memcpy(bfold_sym, d.bfold_sym.data(), sizeof(double) * nr * nr);
    if (bfold_anti && no) std::memcpy(bfold_anti, d.bfold_anti.data(), sizeof(double) * nr * no);
  } catch (const std::exception& ex) {
    return fail(SEM_EINVAL, "sem_axis_fold_host: %s", ex.what());
  }
  return SEM_OK;
}

sem_status sem_plan_create(int k, const int ne[3], const double box[6], double alpha, sem_bc bc, sem_plan** out) {
  const sem_bc bcs[3] = {bc, bc, bc};
  return sem_plan_create_mixed(k, ne, box, alpha, bcs, out);
}

sem_status sem_plan_create_mixed(int k, const int ne[3], const double box[6], double alpha, const sem_bc bc3[3],
                                 sem_plan** out) {
  if (!out || !ne || !box || !bc3) return fail(SEM_EINVAL, "sem_plan_create: null argument");
  *out = nullptr;
  if (k < 1 || k > 64) return fail(SEM_EINVAL, "sem_plan_create: k must be in [1, 64]");
  for (int a = 0; a < 3; ++a)
    if (!valid_bc(bc3[a])) return fail(SEM_EINVAL, "sem_plan_create: bad bc on axis %d", a);
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(SEM_EINVAL, "sem_plan_create: alpha must be finite, >= 0");
  long total = 1;
  for (int a = 0; a < 3; ++a) {
    if (ne[a] < 1) return fail(SEM_EINVAL, "sem_plan_create: ne[%d] < 1", a);
    if (!(box[2 * a] < box[2 * a + 1]) || !std::isfinite(box[2 * a]) || !std::isfinite(box[2 * a + 1]))
      return fail(SEM_EINVAL, "sem_plan_create: degenerate box on axis %d", a);
    const long n = axis_unknowns(bc3[a], ne[a], k);
    if (n < 1) return fail(SEM_EINVAL, "sem_plan_create: Dirichlet axis %d has no interior node", a);
    if (n > 4096) return fail(SEM_EINVAL, "sem_plan_create: axis %d has %ld > 4096 unknowns", a, n);
    total *= n;
  }
  if (total > (1L << 36)) return fail(SEM_EINVAL, "sem_plan_create: problem too large");

  sem_plan* p = new (std::nothrow) sem_plan();
  if (!p) return fail(SEM_ENOMEM, "sem_plan_create: host allocation");
  p->k = k;
  p->alpha = alpha;
  for (int a = 0; a < 3; ++a) {
    p->bc[a] = bc3[a];
    if (bc3[a] == SEM_BC_PERIODIC) p->per_mask |= 1 << a;
  }
  for (int a = 0; a < 6; ++a) p->box[a] = box[a];
  try {
    for (int a = 0; a < 3; ++a) {
      p->ne[a] = ne[a];
      const AxisSpec s = axis_spec(k, ne[a], box[2 * a], box[2 * a + 1], bc3[a]);
      int same = -1;
      for (int b = 0; b < a; ++b)
        if (axis_spec(k, ne[b], box[2 * b], box[2 * b + 1], bc3[b]) == s) same = b;
      if (same >= 0)
        p->ax[a] = p->ax[same];
      else
        build_axis(s, p->ax[a], host_threads());
      p->dims[a] = p->ax[a].n;
    }
  } catch (const std::exception& ex) {
    delete p;
    return fail(SEM_EINVAL, "sem_plan_create: %s", ex.what());
  }
  p->N = (size_t)p->dims[0] * p->dims[1] * p->dims[2];
  const double lmin = p->ax[0].lam[0] + p->ax[1].lam[0] + p->ax[2].lam[0] + alpha;
  const double lmax = p->ax[0].lam.back() + p->ax[1].lam.back() + p->ax[2].lam.back() + alpha;
  if (!(lmin > 1e-13 * lmax)) {
    delete p;
    return fail(SEM_ESINGULAR, "sem_plan_create: operator is singular (min eigenvalue sum %.3e)", lmin);
  }
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "sem_plan_create: no HIP device");
  }
  for (int a = 0; a < 3; ++a) {
    if ((e = upload_fold_factors(p, a)) != hipSuccess) {
      sem_plan_destroy(p);
      return hip_fail(e, "sem_plan_create: folded factor upload");
    }
  }
  for (int a = 0; a < 3; ++a) {
    const int n = p->dims[a];
    p->ld[a] = ((n + 127) / 128) * 128;
    if ((e = upload_factor(p->ax[a].F, n, p->ld[a], &p->d_gf[a])) != hipSuccess ||
        (e = upload_factor(p->ax[a].S, n, p->ld[a], &p->d_gb[a])) != hipSuccess ||
        (e = upload_vec(p->ax[a].lam, &p->d_lam[a])) != hipSuccess ||
        (e = upload_vec(p->ax[a].hband, &p->d_hb[a])) != hipSuccess ||
        (e = upload_vec(p->ax[a].mass, &p->d_mass[a])) != hipSuccess) {
      sem_plan_destroy(p);
      return hip_fail(e, "sem_plan_create: factor upload");
    }
  }
  *out = p;
  return SEM_OK;
}

void sem_plan_destroy(sem_plan* p) {
  if (!p) return;
  int cur = -1;
  (void)hipGetDevice(&cur);
  if (p->device >= 0) (void)hipSetDevice(p->device);
  if (p->stream || p->ws_owned) (void)hipStreamSynchronize(p->stream);
  for (int a = 0; a < 3; ++a) {
    (void)hipFree(p->d_gf[a]);
    (void)hipFree(p->d_gb[a]);
    (void)hipFree(p->d_lam[a]);
    (void)hipFree(p->d_hb[a]);
    (void)hipFree(p->d_mass[a]);
    (void)hipFree(p->d_lamf64[a]);
    for (int b = 0; b < 2; ++b) {
      (void)hipFree(p->d_gff[a][b]);
      (void)hipFree(p->d_gbf[a][b]);
    }
  }
  release_lowp(p);
  if (p->ws_owned) (void)hipFree(p->ws);
  if (cur >= 0) (void)hipSetDevice(cur);
  delete p;
}

sem_status sem_plan_dims(const sem_plan* p, int n[3]) {
  if (!p || !n) return fail(SEM_EINVAL, "sem_plan_dims: null argument");
  for (int a = 0; a < 3; ++a) n[a] = p->dims[a];
  return SEM_OK;
}

sem_status sem_plan_nodes(const sem_plan* p, int axis, double* x) {
  if (!p || !x || axis < 0 || axis > 2) return fail(SEM_EINVAL, "sem_plan_nodes: invalid argument");
  std::memcpy(x, p->ax[axis].x.data(), sizeof(double) * p->dims[axis]);
  return SEM_OK;
}

sem_status sem_plan_eigenvalues(const sem_plan* p, int axis, double* lam) {
  if (!p || !lam || axis < 0 || axis > 2) return fail(SEM_EINVAL, "sem_plan_eigenvalues: invalid argument");
  std::memcpy(lam, p->ax[axis].lam.data(), sizeof(double) * p->dims[axis]);
  return SEM_OK;
}

sem_status sem_plan_set_stream(sem_plan* p, void* s) {
  if (!p) return fail(SEM_EINVAL, "sem_plan_set_stream: null plan");
  p->stream = (hipStream_t)s;
  return SEM_OK;
}

sem_status sem_plan_workspace_bytes(const sem_plan* p, sem_prec prec, size_t* bytes) {
  if (!p || !bytes) return fail(SEM_EINVAL, "sem_plan_workspace_bytes: null argument");
  *bytes = workspace_need(p, prec);
  if (*bytes == 0) return fail(SEM_EINVAL, "sem_plan_workspace_bytes: unknown precision");
  return SEM_OK;
}

sem_status sem_plan_set_workspace(sem_plan* p, void* ptr, size_t bytes) {
  if (!p) return fail(SEM_EINVAL, "sem_plan_set_workspace: null plan");
  if (ptr && ((uintptr_t)ptr % 256) != 0) return fail(SEM_EINVAL, "sem_plan_set_workspace: pointer not 256-B aligned");
  if (p->ws_owned && p->ws) {
    (void)hipStreamSynchronize(p->stream);
    (void)hipFree(p->ws);
  }
  p->ws = ptr;
  p->ws_bytes = ptr ? bytes : 0;
  p->ws_owned = false;
  return SEM_OK;
}

sem_status sem_mode_product(sem_plan* p, int axis, int inverse, const double* in, double* out) {
  if (!p || !in || !out || axis < 0 || axis > 2) return fail(SEM_EINVAL, "sem_mode_product: invalid argument");
  if (in == out) return fail(SEM_EINVAL, "sem_mode_product: in and out must not alias");
  EpiArgs ea;
  hipError_t e = launch_mode_f64(in, out, inverse ? p->d_gb[axis] : p->d_gf[axis], p->ld[axis], p->dims, axis,
                                 EPI_STORE, ea, p->stream);
  if (e != hipSuccess) return hip_fail(e, "sem_mode_product");
  return SEM_OK;
}

sem_status sem_solve(sem_plan* p, const double* f, double* u) {
  if (!p || !f || !u) return fail(SEM_EINVAL, "sem_solve: null argument");
  void* ws = nullptr;
  sem_status st = plan_workspace(p, workspace_need(p, SEM_F64), &ws);
  if (st != SEM_OK) return st;
  hipError_t e = fd64(p, Spectral{p->alpha, 1.0, 0.0}, f, u, (double*)ws);
  if (e != hipSuccess) return hip_fail(e, "sem_solve");
  return SEM_OK;
}

sem_status sem_apply_spectral(sem_plan* p, int kind, double a, double param, const double* f, double* u) {
  if (!p || !f || !u) return fail(SEM_EINVAL, "sem_apply_spectral: null argument");
  if (kind != SEM_SPECTRAL_EXP && kind != SEM_SPECTRAL_POWER)
    return fail(SEM_EINVAL, "sem_apply_spectral: unknown multiplier %d", kind);
  if (!std::isfinite(a) || !std::isfinite(param)) return fail(SEM_EINVAL, "sem_apply_spectral: non-finite parameter");
  if (kind == SEM_SPECTRAL_EXP && param < 0.0) return fail(SEM_EINVAL, "sem_apply_spectral: time must be >= 0");
  const double lmin = p->ax[0].lam[0] + p->ax[1].lam[0] + p->ax[2].lam[0] + a;
  if (kind == SEM_SPECTRAL_POWER && param > 0.0 && !(lmin > 0.0))
    return fail(SEM_ESINGULAR, "sem_apply_spectral: negative power of a singular operator (min L + a = %.3e)", lmin);
  void* ws = nullptr;
  sem_status st = plan_workspace(p, workspace_need(p, SEM_F64), &ws);
  if (st != SEM_OK) return st;
  Spectral sp{a, 1.0, 0.0};
  sp.kind = kind == SEM_SPECTRAL_EXP ? SPECTRAL_EXP : SPECTRAL_POWER;
  sp.param = param;
  hipError_t e = fd64(p, sp, f, u, (double*)ws);
  if (e != hipSuccess) return hip_fail(e, "sem_apply_spectral");
  return SEM_OK;
}

sem_status sem_residual(sem_plan* p, const double* u, const double* f, double* r) {
  if (!p || !u || !f || !r) return fail(SEM_EINVAL, "sem_residual: null argument");
  if (r == u) return fail(SEM_EINVAL, "sem_residual: r must not alias u");
  const double* hb[3] = {p->d_hb[0], p->d_hb[1], p->d_hb[2]};
  ResidualArgs ra;
  ra.periodic = p->per_mask;
  ra.v = u;
  ra.f = f;
  ra.r = r;
  ra.r_kind = 0;
  ra.ldr = p->dims[2];
  ra.cf = 1.0;
  ra.cd = p->alpha;
  ra.ch = 1.0;
  hipError_t e = launch_residual(ra, hb, p->k, p->dims, p->stream);
  if (e != hipSuccess) return hip_fail(e, "sem_residual");
  return SEM_OK;
}

}  // extern "C"
