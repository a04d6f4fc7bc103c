// rowres_inst_split.hip -- row-resident kernels for PATH_SPLIT.
#include "rowres_launch.h"

namespace curob {

hipError_t launch_rowres_split(int kind_hint, const TiledProb &tp, const void *x, void *out, int n, int num_cu,
                            hipStream_t st) {
  return rowres::launch_path<PATH_SPLIT>(kind_hint, tp, x, out, n, num_cu, st, std::make_integer_sequence<int, K_COUNT>{});
}

hipError_t launch_rowres_comp(const void *desc, int nc, int Dpmax, int S, const float *x, int n, int D,
                              const double *o64, const double *sig, const double *lam, const double *cb, double fopt,
                              float *out, int num_cu, hipStream_t st) {
  return rowres::launch_comp(desc, nc, Dpmax, S, x, n, D, o64, sig, lam, cb, fopt, out, num_cu, st);
}

}  // namespace curob
