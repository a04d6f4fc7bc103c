// rowres_inst_split6.hip -- row-resident kernels for PATH_SPLIT6.
#include "rowres_launch.h"

namespace curob {

hipError_t launch_rowres_split6(int kind_hint, const TiledProb &tp, const void *x, void *out, int n, int num_cu,
                            hipStream_t st) {
  return rowres::launch_path<PATH_SPLIT6>(kind_hint, tp, x, out, n, num_cu, st, std::make_integer_sequence<int, K_COUNT>{});
}

}  // namespace curob
