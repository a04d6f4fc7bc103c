// rowres_launch.h -- host side of the row-resident kernel (eval_rowres.h): kernel choice, LDS
// size, persistent grid.
#pragma once

#include <utility>

#include "eval_rowres.h"

namespace curob {

namespace rowres {

// One workgroup per CU (the rows fill most of the LDS): the persistent grid is one workgroup
// per CU, or the tile count when smaller.
inline int persistent_grid(int tiles, int lds_bytes, int num_cu) {
  const int per_cu = kMaxLdsBytes / lds_bytes > 0 ? kMaxLdsBytes / lds_bytes : 1;
  const int cap = num_cu * per_cu;
  const int grid = tiles < cap ? tiles : cap;
  return grid > 0 ? grid : 1;
}

template <int P, int... Ks>
hipError_t launch_path(int kind_hint, const TiledProb &tp, const void *x, void *out, int n, int num_cu,
                       hipStream_t st, std::integer_sequence<int, Ks...>) {
  constexpr int NT = split_terms(P);
  static const void *const basic[] = {reinterpret_cast<const void *>(&k_rowres<NT, Ks>)...};
  // a block of 25..32 m-tiles (a wide hybrid group; basic blocks stay below) takes one pass of
  // four m-tiles per wave instead of two of three
  const bool wide_block = tp.mtiles_max > kPassMTiles && tp.mtiles_max <= kWaves * kMWWide;
  const void *fn = (kind_hint >= 0 && kind_hint < K_COUNT) ? basic[kind_hint]
                   : wide_block ? reinterpret_cast<const void *>(&k_rowres<NT, -1, kMWWide>)
                                : reinterpret_cast<const void *>(&k_rowres<NT, -1>);
  const Carve L = carve(tp.Dp, tp.S, NT);
  if (L.total > kMaxLdsBytes || tp.D > kMaxD) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, L.total);
  if (e != hipSuccess) return e;
  const int grid = persistent_grid((n + kRows - 1) / kRows, L.total, num_cu);
  int wide = (tp.D % 4 == 0 && (reinterpret_cast<uintptr_t>(x) % 16) == 0) ? 1 : 0;
  TiledProb arg = tp;
  const void *xa = x;
  void *oa = out;
  int na = n;
  void *args[] = {&arg, &xa, &na, &oa, &wide};
  return hipLaunchKernel(fn, dim3(grid), dim3(kThreads), args, static_cast<size_t>(L.total), st);
}

// Fused composition: one launch over all rows (desc: device array of nc CompDesc, components
// with pair terms last).
inline hipError_t launch_comp(const void *desc, int nc, int Dpmax, int S, const float *x, int n, int D,
                              const double *o64, const double *sig, const double *lam, const double *cb, double fopt,
                              float *out, int num_cu, hipStream_t st) {
  const void *fn = reinterpret_cast<const void *>(&k_rowres_comp<3>);
  const CompCarve L = comp_carve(Dpmax, S);
  if (L.total > kMaxLdsBytes || D > kMaxD) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, L.total);
  if (e != hipSuccess) return e;
  const int grid = persistent_grid((n + kRows - 1) / kRows, L.total, num_cu);
  int wide = (D % 4 == 0 && (reinterpret_cast<uintptr_t>(x) % 16) == 0) ? 1 : 0;
  const CompDesc *da = static_cast<const CompDesc *>(desc);
  int nca = nc, dpa = Dpmax, sa = S, na = n, dd = D;
  const float *xa = x;
  float *oa = out;
  double fo = fopt;
  void *args[] = {&da, &nca, &dpa, &sa, &xa, &na, &dd, &o64, &sig, &lam, &cb, &fo, &oa, &wide};
  return hipLaunchKernel(fn, dim3(grid), dim3(kThreads), args, static_cast<size_t>(L.total), st);
}

}  // namespace rowres

}  // namespace curob
