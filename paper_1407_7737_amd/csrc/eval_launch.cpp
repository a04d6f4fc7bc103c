// eval_launch.cpp -- host side of the resident kernel: kernel lookup, launch shape, launch.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"
#include "problem.h"

namespace curob {

const void *const *resident_table_split();
const void *const *resident_table_split6();
const void *const *resident_table_f32();
const void *const *resident_table_f64();

namespace {

const void *resident_kernel(int path, int kind, int rot, int vec) {
  if (kind < 0 || kind >= K_COUNT) return nullptr;
  const int idx = (kind * 2 + (rot ? 1 : 0)) * 2 + (vec ? 1 : 0);
  switch (path) {
    case PATH_SPLIT: return resident_table_split()[idx];
    case PATH_SPLIT6: return resident_table_split6()[idx];
    case PATH_F32: return resident_table_f32()[idx];
    case PATH_F64: return resident_table_f64()[idx];
    default: return nullptr;
  }
}

}  // namespace

LaunchShape resident_shape(int path, const DevProb &pb, int n, int num_cu) {
  LaunchShape ls;
  const LdsLayout one = lds_layout(path, pb, 1);
  const int slice = one.total - one.fixed;
  int waves = (kMaxLdsBytes - one.fixed) / slice;
  const int wmax = max_waves_of(path, direct_rows(path, pb.rotated, pb.kind));
  if (waves > wmax) waves = wmax;
  if (waves < 1) waves = 1;
  const int rows = kRowsPerBlock * blocks_of(path);
  const int groups = (n + rows - 1) / rows;
  // small populations: fewer waves per workgroup spread the groups over more CUs
  while (waves > 1 && (groups + waves - 1) / waves < num_cu) waves >>= 1;
  ls.waves = waves;
  ls.lds = lds_layout(path, pb, waves).total;
  int occ = 0;
  const void *fn = resident_kernel(path, pb.kind, pb.rotated, 1);
  if (fn == nullptr ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, 64 * waves, static_cast<size_t>(ls.lds)) != hipSuccess)
    occ = 1;
  if (occ < 1) occ = 1;
  const int need = (groups + waves - 1) / waves;
  const int cap = occ * num_cu;
  ls.grid = need < cap ? (need > 0 ? need : 1) : cap;
  return ls;
}

hipError_t launch_resident(int path, const DevProb &pb, const void *x, void *out, int n, const LaunchShape &ls,
                           hipStream_t st) {
  const size_t esz = path == PATH_F64 ? 8 : 4;
  const int vec = ((pb.D % static_cast<int>(16 / esz)) == 0 && (reinterpret_cast<uintptr_t>(x) % 16) == 0) ? 1 : 0;
  const void *fn = resident_kernel(path, pb.kind, pb.rotated, vec);
  if (fn == nullptr) return hipErrorInvalidValue;
  if (ls.lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, ls.lds);
    if (e != hipSuccess) return e;
  }
  DevProb arg = pb;
  const void *xa = x;
  void *oa = out;
  void *args[] = {&arg, &xa, &oa, &n};
  return hipLaunchKernel(fn, dim3(ls.grid), dim3(64 * ls.waves), args, static_cast<size_t>(ls.lds), st);
}

}  // namespace curob
