// Internal to the library: the context structure and the solver entry points
// that the warm-start network's translation unit calls.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <functional>

#include "alloc.h"

struct alloc_ctx {
  int device;
  hipStream_t stream;
  char* ws;  // device workspace of the solver
  size_t ws_bytes;
  int cus;
  size_t lds_max;
  int timing;
  hipEvent_t ev0, ev1;
  double last_ms;
  int refs;    // live batches and networks made on this context
  int closed;  // alloc_ctx_destroy was called while refs > 0: freed with the last of them
  char* scratch;  // device address of the library's fixed workspace on this device
};

namespace alloc_internal {

// A batch or network made on the context holds it; the context is freed when
// it was destroyed and its last holder goes.
void ctx_retain(alloc_ctx* c);
void ctx_release(alloc_ctx* c);

// A warm start held in device memory (float64); any pointer may be null.
struct DevWarm {
  const double* p0;     // [M][N][K]
  const double* xi0;    // [M]
  const double* zeta0;  // [K]
};

// Produces drop b's warm start on the context's stream.  Returns 0 or a
// negative code; leaving every pointer null means a cold start.
using WarmFn = std::function<int(int b, DevWarm* out)>;

// alloc_solve with the warm start in device memory (dev may be null).
int solve_one(alloc_ctx* ctx, const alloc_problem* pb, const alloc_params* prm, const alloc_warm* host,
              const DevWarm* dev, alloc_result* res);
// The same on a fixed device workspace of fixed_bytes (fixed != null): a
// layout that does not fit is rejected with ALLOC_ETOOBIG.
int solve_one_ws(alloc_ctx* ctx, const alloc_problem* pb, const alloc_params* prm, const alloc_warm* host,
                 const DevWarm* dev, alloc_result* res, char* fixed, size_t fixed_bytes);

// alloc_solve_batch with warm starts from host arrays (host, [B] or null) or
// from a producer (fn, or null).
int solve_batch(alloc_ctx* ctx, int B, const alloc_problem* probs, const alloc_params* prm,
                const alloc_warm* host, const WarmFn* fn, alloc_result* results);

}  // namespace alloc_internal
