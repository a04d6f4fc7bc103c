// tiled_inst_split6.hip -- tiled-path kernels for PATH_SPLIT6.
#include "eval_tiled.h"

namespace curob {

hipError_t launch_tiled_split6(int kind_hint, const TiledProb &tp, const void *x, void *out, int n, int cap,
                         void *partials, void *zbuf, void *pack, hipStream_t st) {
  return tiled::launch_tiled_path<PATH_SPLIT6>(kind_hint, tp, x, out, n, cap, partials, zbuf, pack, st,
                                          std::make_integer_sequence<int, K_COUNT>{});
}

}  // namespace curob
