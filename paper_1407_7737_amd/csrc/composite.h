// composite.h -- hybrid (Sec. 5) and composition (Sec. 6) evaluation, and basic functions of
// dimension above the resident kernel's range.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "problem.h"

namespace curob {

struct CompositeDev {
  std::vector<void *> allocs;
  bool ready = false;
  void release();
};

// Uploads whatever the composite kernels need for p (nothing for small basic problems).
hipError_t build_composite(const Problem &p, CompositeDev &cd);

// Evaluates n rows of x into out on the given path.
hipError_t launch_composite(int path, const CompositeDev &cd, const void *x, void *out, int n, int num_cu,
                            hipStream_t st);

}  // namespace curob
