// FP64 fast-diagonalisation solve that allocates nothing.
//
// sem_solve keeps its one intermediate array (N doubles between the mode
// products) in the plan workspace, which it allocates on first use unless the
// caller installed one.  sem_solve_noalloc runs the same mode products with that
// array in a fixed device array of this library instead, so that callers that
// cannot allocate (code under stream capture, tight serving loops, allocation-
// free harnesses) can solve without any hipMalloc.  Each device that runs it
// holds its own copy of the array for the life of the process; the host-side
// name of the array is only a handle, its device address is looked up once per
// device with hipGetSymbolAddress.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.h"
#include "plan_internal.h"

namespace semfd {
namespace {

constexpr size_t kScratchDoubles = SEM_NOALLOC_MAX_UNKNOWNS;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (the current device is the
// plan's), looked up on the first call per device.
sem_status scratch_for_device(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) return set_error(SEM_EINVAL, "sem_solve_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "sem_solve_noalloc: scratch address");
    if (!ptr) return set_error(SEM_EDEVICE, "sem_solve_noalloc: scratch address is null");
    g_scratch_ptr[device] = (double*)ptr;
  }
  *out = g_scratch_ptr[device];
  return SEM_OK;
}

}  // namespace
}  // namespace semfd

using namespace semfd;

extern "C" sem_status sem_solve_noalloc(sem_plan* p, const double* f, double* u) {
  if (!p || !f || !u) return set_error(SEM_EINVAL, "sem_solve_noalloc: null argument");
  if (p->N > kScratchDoubles)
    return set_error(SEM_EINVAL, "sem_solve_noalloc: more unknowns than the fixed scratch array holds "
                                 "(SEM_NOALLOC_MAX_UNKNOWNS)");
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "sem_solve_noalloc: current device");
  if (cur != p->device && (e = hipSetDevice(p->device)) != hipSuccess) return hip_fail(e, "sem_solve_noalloc: device");
  double* tmp = nullptr;
  sem_status st = scratch_for_device(p->device, &tmp);
  if (st == SEM_OK) {
    e = fd64(p, Spectral{p->alpha, 1.0, 0.0}, f, u, tmp);
    if (e != hipSuccess) st = hip_fail(e, "sem_solve_noalloc");
  }
  if (cur != p->device) (void)hipSetDevice(cur);
  return st;
}
