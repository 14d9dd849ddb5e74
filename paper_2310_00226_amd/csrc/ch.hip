// Cahn-Hilliard IMEX time stepping (paper Sec. 3.6, eq. chscheme-2) on the
// fast-diagonalisation solver, one HIP graph per step.
//
// The scheme (BDF2 with an explicit extrapolation of the nonlinear term):
//   a phi_{n+1} - m dt Lap w_{n+1} = phi_hat,   w_{n+1} = -eps Lap phi_{n+1} + (1/eps) F'(phi_bar)
//   a = 3/2, phi_hat = 2 phi_n - phi_{n-1}/2, phi_bar = 2 phi_n - phi_{n-1},
//   F'(phi) = phi^3 - phi,
// with the discrete Laplacian Lap_h = -H_3 = -(H_x + H_y + H_z), H = M^{-1} K per
// axis (homogeneous Neumann: natural boundary condition, all nodes unknown).
// Eliminating w gives one linear system per step,
//   (a I + m dt eps H_3^2) phi_{n+1} = phi_hat - (m dt / eps) H_3 g,   g = F'(phi_bar),
// which the eigen-decomposition diagonalises: H_3 = S_3 Lambda3D S_3^{-1}, so
//   phi_{n+1} = S_3 [ (S_3^{-1} rhs) / (a + m dt eps Lambda3D^2) ].
// The paper applies this as a two-right-hand-side transform of phi_hat and g with
// Lambda3D g~ formed in the eigenbasis; here the H_3 g term is applied matrix-free
// in FP64 to form rhs (identical in exact arithmetic, three mode products fewer),
// then one FD application in the chosen precision gives phi_{n+1}, and
// `refine_sweeps` FP64 iterative-refinement sweeps against the operator
// a I + c H_3^2 (c = m dt eps), each
//   w = H_3 phi,  r = rhs - a phi - c H_3 w,  phi += FD(r),
// recover FP64 accuracy.
//
// Per step: one pointwise kernel, one banded pass for rhs, one FD application
// (six mode products) and per sweep two banded passes + one FD application.  The
// whole step is captured once per buffer rotation phase into a HIP graph and
// replayed; three phases rotate (phi_{n-1}, phi_n, phi_{n+1}) through the caller's
// two arrays and one internal array.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>

#include "kernels.h"
#include "plan_internal.h"

struct sem_ch {
  sem_plan* plan = nullptr;
  double eps = 0, mob = 0, dt = 0, a = 1.5;
  sem_prec prec = SEM_F32;
  int sweeps = 0;
  size_t N = 0;
  hipStream_t stream = nullptr;       // own stream (graph capture needs a non-null stream)
  hipStream_t user_stream = nullptr;  // caller's stream (ordering only)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  double* phi3 = nullptr;  // third time level
  double* phat = nullptr;  // phi_hat; FP64 correction in FP64 mode
  double* g = nullptr;     // F'(phi_bar); FP64 residual in FP64 mode
  double* rhs = nullptr;
  double* w = nullptr;     // H_3 phi during sweeps
  semfd::LpWork lw;
  double* tmp64 = nullptr;  // FP64 FD scratch (plan workspace) in FP64 mode
  const double* forcing = nullptr;  // optional source s at t_{n+1} (caller-owned)
  int use_graphs = 1;
  hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
  const double* key_n = nullptr;
  const double* key_nm1 = nullptr;
};

namespace semfd {
namespace {

__global__ __launch_bounds__(256) void ch_pointwise_kernel(const double* __restrict__ cur,
                                                           const double* __restrict__ prev, double* __restrict__ phat,
                                                           double* __restrict__ g, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double c = cur[i], p = prev[i];
    phat[i] = 2.0 * c - 0.5 * p;
    const double b = 2.0 * c - p;
    g[i] = b * b * b - b;
  }
}

__global__ __launch_bounds__(256) void axpy_kernel(double* __restrict__ u, const double* __restrict__ d, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    u[i] += d[i];
}

unsigned grid_for(size_t n) {
  const size_t b = (n + 255) / 256;
  return (unsigned)(b < 16384 ? (b > 0 ? b : 1) : 16384);
}

void drop_graphs(sem_ch* c) {
  for (int i = 0; i < 3; ++i) {
    if (c->exec[i]) (void)hipGraphExecDestroy(c->exec[i]);
    c->exec[i] = nullptr;
  }
  c->key_n = c->key_nm1 = nullptr;
}

// All work of one step on c->stream: prev = phi_{n-1}, cur = phi_n -> next = phi_{n+1}.
hipError_t enqueue_step(sem_ch* c, const double* prev, const double* cur, double* next) {
  sem_plan* p = c->plan;
  const double* hb[3] = {p->d_hb[0], p->d_hb[1], p->d_hb[2]};
  const double cH = c->mob * c->dt * c->eps;
  const Spectral sp{c->a, 0.0, cH};
  hipError_t e;
  ch_pointwise_kernel<<<grid_for(c->N), 256, 0, c->stream>>>(cur, prev, c->phat, c->g, c->N);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  {  // rhs = phi_hat (+ dt s) - (m dt / eps) H_3 g
    ResidualArgs ra;
    ra.v = c->g;
    ra.f = c->phat;
    ra.r = c->rhs;
    ra.r_kind = 0;
    ra.ldr = p->dims[2];
    ra.cf = 1.0;
    ra.cd = 0.0;
    if (c->forcing) {  // BDF2 for phi_t = m Lap mu + s: the source enters as dt s
      ra.d = c->forcing;
      ra.cd = -c->dt;
    }
    ra.ch = c->mob * c->dt / c->eps;
    if ((e = launch_residual(ra, hb, p->k, p->dims, c->stream)) != hipSuccess) return e;
  }
  const bool f64 = c->prec == SEM_F64;
  if (f64)
    e = fd64(p, sp, c->rhs, next, c->tmp64);
  else
    e = lp_fd(p, c->lw, sp, c->rhs, next, 1, nullptr);
  if (e != hipSuccess) return e;
  for (int s = 0; s < c->sweeps; ++s) {
    ResidualArgs hw;  // w = H_3 phi
    hw.v = next;
    hw.r = c->w;
    hw.r_kind = 0;
    hw.ldr = p->dims[2];
    hw.cf = 0.0;
    hw.cd = 0.0;
    hw.ch = -1.0;
    if ((e = launch_residual(hw, hb, p->k, p->dims, c->stream)) != hipSuccess) return e;
    ResidualArgs rr;  // r = rhs - a phi - c H_3 w
    rr.v = c->w;
    rr.f = c->rhs;
    rr.d = next;
    rr.cf = 1.0;
    rr.cd = c->a;
    rr.ch = cH;
    if (f64) {
      rr.r = c->g;
      rr.r_kind = 0;
      rr.ldr = p->dims[2];
    } else {
      rr.r = c->lw.r;
      rr.r_kind = c->lw.rkind;
      rr.ldr = c->lw.ldr;
      rr.rplane = c->lw.rplane;
    }
    if ((e = launch_residual(rr, hb, p->k, p->dims, c->stream)) != hipSuccess) return e;
    if (f64) {
      if ((e = fd64(p, sp, c->g, c->phat, c->tmp64)) != hipSuccess) return e;
      axpy_kernel<<<grid_for(c->N), 256, 0, c->stream>>>(next, c->phat, c->N);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    } else if ((e = lp_fd(p, c->lw, sp, nullptr, next, 0, nullptr)) != hipSuccess) {
      return e;
    }
  }
  return hipSuccess;
}

sem_status capture(sem_ch* c, int phase, double* const buf[3]) {
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "sem_ch_step: begin capture");
  const hipError_t ek = enqueue_step(c, buf[phase % 3], buf[(phase + 1) % 3], buf[(phase + 2) % 3]);
  e = hipStreamEndCapture(c->stream, &graph);
  if (ek != hipSuccess || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_fail(ek != hipSuccess ? ek : e, "sem_ch_step: capture");
  }
  e = hipGraphInstantiate(&c->exec[phase], graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    c->exec[phase] = nullptr;
    return hip_fail(e, "sem_ch_step: graph instantiate");
  }
  return SEM_OK;
}

}  // namespace
}  // namespace semfd

using namespace semfd;

extern "C" {

void sem_ch_destroy(sem_ch* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);
  (void)hipFree(c->phi3);
  (void)hipFree(c->phat);
  (void)hipFree(c->g);
  (void)hipFree(c->rhs);
  (void)hipFree(c->w);
  if (c->ev_in) (void)hipEventDestroy(c->ev_in);
  if (c->ev_out) (void)hipEventDestroy(c->ev_out);
  sem_plan_destroy(c->plan);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

sem_status sem_ch_create(int k, const int ne[3], const double box[6], double eps, double mob, double dt,
                         sem_prec prec, int refine_sweeps, sem_ch** out) {
  if (!out) return set_error(SEM_EINVAL, "sem_ch_create: null output");
  *out = nullptr;
  if (!(eps > 0) || !(mob > 0) || !(dt > 0) || !std::isfinite(eps) || !std::isfinite(mob) || !std::isfinite(dt))
    return set_error(SEM_EINVAL, "sem_ch_create: eps, mobility and dt must be positive and finite");
  if (refine_sweeps < 0 || refine_sweeps > 64) return set_error(SEM_EINVAL, "sem_ch_create: refine_sweeps in [0, 64]");
  if (prec != SEM_F64 && prec != SEM_F32 && prec != SEM_BF16 && prec != SEM_BF16X3)
    return set_error(SEM_EINVAL, "sem_ch_create: unknown precision");
  sem_ch* c = new (std::nothrow) sem_ch;
  if (!c) return set_error(SEM_ENOMEM, "sem_ch_create: host allocation");
  c->eps = eps;
  c->mob = mob;
  c->dt = dt;
  c->prec = prec;
  c->sweeps = refine_sweeps;
  // the plan's alpha is the BDF2 coefficient a (positive: no singular mode)
  sem_status st = sem_plan_create(k, ne, box, c->a, SEM_BC_NEUMANN, &c->plan);
  if (st != SEM_OK) {
    delete c;
    return st;
  }
  c->N = c->plan->N;
  hipError_t e;
  if ((e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming)) != hipSuccess) {
    sem_ch_destroy(c);
    return hip_fail(e, "sem_ch_create: stream / events");
  }
  c->plan->stream = c->stream;
  const size_t bytes = c->N * sizeof(double);
  if ((e = hipMalloc(&c->phi3, bytes)) != hipSuccess || (e = hipMalloc(&c->phat, bytes)) != hipSuccess ||
      (e = hipMalloc(&c->g, bytes)) != hipSuccess || (e = hipMalloc(&c->rhs, bytes)) != hipSuccess ||
      (e = hipMalloc(&c->w, bytes)) != hipSuccess) {
    sem_ch_destroy(c);
    return e == hipErrorOutOfMemory ? set_error(SEM_ENOMEM, "sem_ch_create: device allocation")
                                    : hip_fail(e, "sem_ch_create: device allocation");
  }
  // everything a step needs is allocated now, so that steps can be captured
  if (prec == SEM_F64) {
    void* ws = nullptr;
    st = plan_workspace(c->plan, workspace_need(c->plan, SEM_F64), &ws);
    c->tmp64 = (double*)ws;
  } else {
    st = lp_prepare(c->plan, prec, &c->lw);
  }
  if (st != SEM_OK) {
    sem_ch_destroy(c);
    return st;
  }
  *out = c;
  return SEM_OK;
}

sem_status sem_ch_dims(const sem_ch* c, int n[3]) {
  if (!c || !n) return set_error(SEM_EINVAL, "sem_ch_dims: null argument");
  return sem_plan_dims(c->plan, n);
}

sem_status sem_ch_tuning(const sem_ch* c, int* tuned, int choice[6]) {
  if (!c || !tuned || !choice) return set_error(SEM_EINVAL, "sem_ch_tuning: null argument");
  if (c->prec == SEM_F64) {  // FP64 mode products have no tunable shape
    *tuned = 0;
    for (int s = 0; s < 6; ++s) choice[s] = 0;
    return SEM_OK;
  }
  return sem_plan_tuning(c->plan, c->prec, tuned, choice);
}

sem_status sem_ch_set_stream(sem_ch* c, void* s) {
  if (!c) return set_error(SEM_EINVAL, "sem_ch_set_stream: null handle");
  c->user_stream = (hipStream_t)s;
  return SEM_OK;
}

sem_status sem_ch_set_graphs(sem_ch* c, int enable) {
  if (!c) return set_error(SEM_EINVAL, "sem_ch_set_graphs: null handle");
  c->use_graphs = enable ? 1 : 0;
  return SEM_OK;
}

sem_status sem_ch_set_forcing(sem_ch* c, const double* s) {
  if (!c) return set_error(SEM_EINVAL, "sem_ch_set_forcing: null handle");
  if (s != c->forcing) drop_graphs(c);  // the captured steps hold the old pointer
  c->forcing = s;
  return SEM_OK;
}

sem_status sem_ch_step(sem_ch* c, double* phi_n, double* phi_nm1, int nsteps) {
  if (!c || !phi_n || !phi_nm1 || nsteps < 0) return set_error(SEM_EINVAL, "sem_ch_step: invalid argument");
  if (phi_n == phi_nm1) return set_error(SEM_EINVAL, "sem_ch_step: phi_n and phi_nm1 must be distinct arrays");
  if (nsteps == 0) return SEM_OK;
  double* const buf[3] = {phi_nm1, phi_n, c->phi3};
  if (c->use_graphs && (c->key_n != phi_n || c->key_nm1 != phi_nm1 || !c->exec[0])) {
    drop_graphs(c);
    for (int ph = 0; ph < 3; ++ph) {
      sem_status st = capture(c, ph, buf);
      if (st != SEM_OK) {
        drop_graphs(c);
        return st;
      }
    }
    c->key_n = phi_n;
    c->key_nm1 = phi_nm1;
  }
  hipError_t e;
  if ((e = hipEventRecord(c->ev_in, c->user_stream)) != hipSuccess ||
      (e = hipStreamWaitEvent(c->stream, c->ev_in, 0)) != hipSuccess)
    return hip_fail(e, "sem_ch_step: stream ordering");
  for (int s = 0; s < nsteps; ++s) {
    const int ph = s % 3;
    if (c->use_graphs)
      e = hipGraphLaunch(c->exec[ph], c->stream);
    else
      e = enqueue_step(c, buf[ph], buf[(ph + 1) % 3], buf[(ph + 2) % 3]);
    if (e != hipSuccess) return hip_fail(e, "sem_ch_step: step");
  }
  // after nsteps the levels sit at prev = buf[nsteps % 3], cur = buf[(nsteps + 1) % 3];
  // move them back into the caller's arrays (phi_nm1 = buf[0], phi_n = buf[1])
  const size_t bytes = c->N * sizeof(double);
  const int rot = nsteps % 3;
  if (rot == 1) {  // prev = phi_n array, cur = internal
    if ((e = hipMemcpyAsync(phi_nm1, phi_n, bytes, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(phi_n, c->phi3, bytes, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)
      return hip_fail(e, "sem_ch_step: rotate");
  } else if (rot == 2) {  // prev = internal, cur = phi_nm1 array
    if ((e = hipMemcpyAsync(phi_n, phi_nm1, bytes, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(phi_nm1, c->phi3, bytes, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)
      return hip_fail(e, "sem_ch_step: rotate");
  }
  if ((e = hipEventRecord(c->ev_out, c->stream)) != hipSuccess ||
      (e = hipStreamWaitEvent(c->user_stream, c->ev_out, 0)) != hipSuccess)
    return hip_fail(e, "sem_ch_step: stream ordering");
  return SEM_OK;
}

}  // extern "C"
