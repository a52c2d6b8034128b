// dirac_batch.hip -- batches of independent instances (filled in with the
// batched launch).
#include "dirac_plan.h"

using namespace dirac;

extern "C" int dl_batch_create(dl_plan* out, const dl_grid*, const double*, const double*,
                               const double*, const double*, int, dl_dtype, dl_bc, unsigned) {
  if (out) *out = nullptr;
  return set_error(DL_ERR_STATE, "batches not available in this build");
}
extern "C" int dl_batch_step(dl_plan, void* const*, const double* const*, const int64_t*, void*) {
  return set_error(DL_ERR_STATE, "batches not available in this build");
}
