// Workspace sizing and (later) the mixed-precision paths.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "plan_internal.h"

namespace semfd {

size_t workspace_need(const sem_plan* p, sem_prec prec) {
  const size_t n = p->N;
  switch (prec) {
    case SEM_F64:
      return ((n * sizeof(double) + 255) / 256) * 256;
    default:
      return 0;
  }
}

void release_lowp(sem_plan*) {}

}  // namespace semfd
