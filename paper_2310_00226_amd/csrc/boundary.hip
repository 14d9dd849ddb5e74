// Non-homogeneous boundary data moved into the right-hand side (paper Sec. 2.1
// remark: Dirichlet values and Neumann fluxes enter the right-hand side, the
// matrix to invert stays the same), sem_lift_boundary.
//
// Per axis a, the face data g_lo (x_a = lower end) and g_hi (upper end) are
// arrays over the two other axes.  Each thread owns one line along a through the
// face point and adds  c_lo[d] g_lo  at unknown d and  c_hi[d] g_hi  at unknown
// n_a - 1 - d, d < depth (Dirichlet: c = -H(unknown, removed end node) of the
// full-grid assembly, depth = min(k, n_a); Neumann: c = 1 / M_a(end), depth 1).
// A thread does both ends of its line in order, so lines shorter than 2 depth
// need no synchronisation; the three axes are three launches on one stream.
#include <hip/hip_runtime.h>

#include "../../include/sem.h"
#include "kernels.h"
#include "plan_internal.h"

namespace semfd {
namespace {

constexpr int MAX_DEPTH = 64;  // k <= 64

struct LiftCoef {
  double lo[MAX_DEPTH], hi[MAX_DEPTH];
};

__global__ __launch_bounds__(256) void lift_face_kernel(double* __restrict__ f, const double* __restrict__ glo,
                                                        const double* __restrict__ ghi, LiftCoef c, int depth, int n,
                                                        long sa, int m2, long s1, long s2, long count) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const long p = t / m2, q = t - p * m2;
  const long base = p * s1 + q * s2;
  const double vlo = glo ? glo[t] : 0.0;
  const double vhi = ghi ? ghi[t] : 0.0;
  for (int d = 0; d < depth; ++d) {
    if (glo) f[base + (long)d * sa] += c.lo[d] * vlo;
    if (ghi) f[base + (long)(n - 1 - d) * sa] += c.hi[d] * vhi;
  }
}

bool overlaps(const double* a, size_t na, const double* b, size_t nb) {
  const char *a0 = (const char*)a, *b0 = (const char*)b;
  return a0 < b0 + nb * sizeof(double) && b0 < a0 + na * sizeof(double);
}

}  // namespace
}  // namespace semfd

using namespace semfd;

extern "C" sem_status sem_lift_boundary(sem_plan* p, const double* const g[6], double* f) {
  if (!p || !f) return set_error(SEM_EINVAL, "sem_lift_boundary: null argument");
  if (!g) return SEM_OK;
  const int* n = p->dims;
  const long plane = (long)n[1] * n[2];
  // strides of the three axes; the face of axis a spans the two others in order
  const long stride[3] = {plane, (long)n[2], 1};
  for (int a = 0; a < 3; ++a) {
    const double* lo = g[2 * a];
    const double* hi = g[2 * a + 1];
    if (!lo && !hi) continue;
    if (p->bc[a] == SEM_BC_PERIODIC)
      return set_error(SEM_EINVAL, "sem_lift_boundary: a periodic axis has no boundary data");
    const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
    const long count = (long)n[b1] * n[b2];
    if ((lo && overlaps(lo, count, f, p->N)) || (hi && overlaps(hi, count, f, p->N)))
      return set_error(SEM_EINVAL, "sem_lift_boundary: face data must not alias f");
  }
  for (int a = 0; a < 3; ++a) {
    const double* lo = g[2 * a];
    const double* hi = g[2 * a + 1];
    if (!lo && !hi) continue;
    const AxisData& ax = p->ax[a];
    const int depth = (int)ax.lift_lo.size();
    if (depth < 1 || depth > MAX_DEPTH || ax.lift_hi.size() != ax.lift_lo.size())
      return set_error(SEM_EINVAL, "sem_lift_boundary: plan has no boundary coupling");
    LiftCoef c{};
    for (int d = 0; d < depth; ++d) {
      c.lo[d] = ax.lift_lo[d];
      c.hi[d] = ax.lift_hi[d];
    }
    const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
    const long count = (long)n[b1] * n[b2];
    const unsigned blocks = (unsigned)((count + 255) / 256);
    lift_face_kernel<<<blocks, 256, 0, p->stream>>>(f, lo, hi, c, depth, n[a], stride[a], n[b2], stride[b1],
                                                     stride[b2], count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "sem_lift_boundary");
  }
  return SEM_OK;
}
