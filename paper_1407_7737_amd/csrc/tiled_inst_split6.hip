// tiled_inst_split6.hip -- tiled-path kernels for PATH_SPLIT6.
#include <utility>

#include "eval_tiled.h"

namespace curob {

namespace {
template <int... Ks>
const void *const *partial_table(std::integer_sequence<int, Ks...>) {
  static const void *const tab[] = {reinterpret_cast<const void *>(&tiled::k_tiled_partial<PATH_SPLIT6, Ks>)...};
  return tab;
}
}  // namespace

hipError_t launch_tiled_split6(int kind_hint, const TiledProb &tp, const void *x, void *out, int n, void *partials,
                         void *zbuf, hipStream_t st) {
  const void *fn = (kind_hint >= 0 && kind_hint < K_COUNT)
                       ? partial_table(std::make_integer_sequence<int, K_COUNT>{})[kind_hint]
                       : reinterpret_cast<const void *>(&tiled::k_tiled_partial<PATH_SPLIT6, -1>);
  TiledProb arg = tp;
  const void *xa = x;
  void *pa = partials, *za = zbuf, *oa = out;
  int na = n;
  void *args[] = {&arg, &xa, &na, &pa, &za};
  hipError_t e = hipLaunchKernel(fn, dim3(tp.ngroups, (n + kTileRows - 1) / kTileRows), dim3(256), args, 0, st);
  if (e != hipSuccess) return e;
  void *fargs[] = {&arg, &pa, &za, &na, &oa};
  return hipLaunchKernel(reinterpret_cast<const void *>(&tiled::k_tiled_finalize<PATH_SPLIT6>), dim3((n + 3) / 4),
                         dim3(256), fargs, 0, st);
}

}  // namespace curob
