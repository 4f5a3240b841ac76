// Test harness for the solver's double-precision logarithms (csrc/logs.h):
// evaluates one of them on n host values on the GPU and copies the results
// back.  Built beside the tests; the solver library does not contain it.
#include <hip/hip_runtime.h>

#include "logs.h"

namespace {

__global__ void eval_kernel(const double* x, double* y, int n, int which) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = x[i];
  double r;
  switch (which) {
    case 0: r = alloc_logs::log_d(v); break;
    case 1: r = alloc_logs::log1p_d(v); break;
    case 2: r = alloc_logs::log2_d(v); break;
    default: r = alloc_logs::log2_1p_d(v); break;
  }
  y[i] = r;
}

}  // namespace

// which: 0 log, 1 log1p, 2 log2, 3 log2(1 + x).  Returns 0, or -1 on a HIP
// error, -2 on bad arguments.
extern "C" __attribute__((visibility("default"))) int logs_probe_eval(const double* x, double* y, int n,
                                                                       int which) {
  if (!x || !y || n < 1 || which < 0 || which > 3) return -2;
  double *dx = nullptr, *dy = nullptr;
  const size_t bytes = sizeof(double) * (size_t)n;
  int rc = 0;
  if (hipMalloc((void**)&dx, bytes) != hipSuccess || hipMalloc((void**)&dy, bytes) != hipSuccess) rc = -1;
  if (!rc && hipMemcpy(dx, x, bytes, hipMemcpyHostToDevice) != hipSuccess) rc = -1;
  if (!rc) {
    hipLaunchKernelGGL(eval_kernel, dim3((n + 255) / 256), dim3(256), 0, 0, dx, dy, n, which);
    if (hipGetLastError() != hipSuccess || hipMemcpy(y, dy, bytes, hipMemcpyDeviceToHost) != hipSuccess) rc = -1;
  }
  if (dx) (void)hipFree(dx);
  if (dy) (void)hipFree(dy);
  return rc;
}
