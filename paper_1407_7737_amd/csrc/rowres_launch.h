// rowres_launch.h -- host side of the row-resident kernel (eval_rowres.h): kernel choice, LDS
// size, persistent grid.
#pragma once

#include <utility>

#include "eval_rowres.h"

namespace curob {

namespace rowres {

// 16-row column blocks per workgroup: two, or one when pair terms need the z copy in LDS.
inline int column_blocks(int kind_hint, const TiledProb &tp) {
  const bool pairs = kind_hint >= 0 ? kind_is_pairwise(kind_hint) : tp.any_pairwise != 0;
  return pairs ? 1 : 2;
}

template <int P, int... Ks>
hipError_t launch_path(int kind_hint, const TiledProb &tp, const void *x, void *out, int n, int num_cu,
                       hipStream_t st, std::integer_sequence<int, Ks...>) {
  static const void *const basic[] = {
      reinterpret_cast<const void *>(&k_rowres<P, Ks, KindTraits<Ks>::pairwise ? 1 : 2>)...};
  const int CB = column_blocks(kind_hint, tp);
  const void *fn;
  if (kind_hint >= 0 && kind_hint < K_COUNT) fn = basic[kind_hint];
  else fn = CB == 1 ? reinterpret_cast<const void *>(&k_rowres<P, -1, 1>) : reinterpret_cast<const void *>(&k_rowres<P, -1, 2>);
  const Carve L = carve(tp.Dp, tp.S, CB, CB == 1);
  if (L.total > kMaxLdsBytes) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, L.total);
  if (e != hipSuccess) return e;
  const int R = 16 * CB;
  const int tiles = (n + R - 1) / R;
  const int per_cu = kMaxLdsBytes / L.total > 0 ? kMaxLdsBytes / L.total : 1;
  const int cap = num_cu * per_cu;
  const int grid = tiles < cap ? tiles : cap;
  int wide = (tp.D % 4 == 0 && (reinterpret_cast<uintptr_t>(x) % 16) == 0) ? 1 : 0;
  TiledProb arg = tp;
  const void *xa = x;
  void *oa = out;
  int na = n;
  void *args[] = {&arg, &xa, &na, &oa, &wide};
  return hipLaunchKernel(fn, dim3(grid > 0 ? grid : 1), dim3(kThreads), args, static_cast<size_t>(L.total), st);
}

// Fused composition: one launch over all rows (desc: device array of nc CompDesc).
inline hipError_t launch_comp(const void *desc, int nc, int Dpmax, int S, int CB, const float *x, int n, int D,
                              const double *o64, const double *sig, const double *lam, const double *cb, double fopt,
                              float *out, int num_cu, hipStream_t st) {
  const void *fn = CB == 1 ? reinterpret_cast<const void *>(&k_rowres_comp<1>)
                           : reinterpret_cast<const void *>(&k_rowres_comp<2>);
  const CompCarve L = comp_carve(Dpmax, S, CB);
  if (L.total > kMaxLdsBytes) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, L.total);
  if (e != hipSuccess) return e;
  const int R = 16 * CB;
  const int tiles = (n + R - 1) / R;
  const int per_cu = kMaxLdsBytes / L.total > 0 ? kMaxLdsBytes / L.total : 1;
  const int cap = num_cu * per_cu;
  const int grid = tiles < cap ? tiles : cap;
  int wide = (D % 4 == 0 && (reinterpret_cast<uintptr_t>(x) % 16) == 0) ? 1 : 0;
  const CompDesc *da = static_cast<const CompDesc *>(desc);
  int nca = nc, dpa = Dpmax, sa = S, na = n, dd = D;
  const float *xa = x;
  float *oa = out;
  double fo = fopt;
  void *args[] = {&da, &nca, &dpa, &sa, &xa, &na, &dd, &o64, &sig, &lam, &cb, &fo, &oa, &wide};
  return hipLaunchKernel(fn, dim3(grid > 0 ? grid : 1), dim3(kThreads), args, static_cast<size_t>(L.total), st);
}

}  // namespace rowres

}  // namespace curob
