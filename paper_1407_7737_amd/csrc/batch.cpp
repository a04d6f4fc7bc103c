// batch.cpp -- batched populations (one persistent launch, HIP graph replay).
#include <hip/hip_runtime.h>

#include "../../include/curob.h"

extern "C" {
int curob_batch_create(int, const int *, const int *, const int *, unsigned long long, curob_batch **out) {
  if (out) *out = nullptr;
  return CUROB_E_ARG;
}
int curob_batch_bind(curob_batch *, const float *const *, float *const *) { return CUROB_E_ARG; }
int curob_batch_run(curob_batch *) { return CUROB_E_ARG; }
int curob_batch_destroy(curob_batch *) { return CUROB_OK; }
}
