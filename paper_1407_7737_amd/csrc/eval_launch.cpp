// eval_launch.cpp -- host side of the resident kernel: kernel lookup, launch shape, launch.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <tuple>

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

std::map<std::tuple<int, int, int, int>, std::pair<int, int>> &overrides() {
  static std::map<std::tuple<int, int, int, int>, std::pair<int, int>> m;
  return m;
}

// waves (already legal) -> shape: LDS of that many slices, grid of at most occupancy x CUs
// workgroups (grid_per8 > 0: at most that many per 8 CUs), no more than the row groups need
LaunchShape shape_with(int path, const DevProb &pb, int n, int num_cu, int waves, int grid_per8) {
  LaunchShape ls;
  const int rows = kRowsPerBlock * blocks_of(path);
  const int groups = (n + rows - 1) / rows;
  ls.waves = waves;
  ls.lds = lds_layout(path, pb, waves).total;
  int occ = 0;
  const void *fn = resident_kernel(path, pb.kind, pb.rotated, 1);
  if (fn == nullptr ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, 64 * waves, static_cast<size_t>(ls.lds)) != hipSuccess)
    occ = 1;
  if (occ < 1) occ = 1;
  const int need = (groups + waves - 1) / waves;
  int cap = occ * num_cu;
  if (grid_per8 > 0) {
    const int want = (grid_per8 * num_cu + 7) / 8;
    if (want < cap) cap = want > 0 ? want : 1;
  }
  ls.grid = need < cap ? (need > 0 ? need : 1) : cap;
  return ls;
}

}  // namespace

int resident_max_waves(int path, const DevProb &pb) {
  const LdsLayout one = lds_layout(path, pb, 1);
  const int slice = one.total - one.fixed;
  int waves = (kMaxLdsBytes - one.fixed) / slice;
  const int wmax = max_waves_of(path, direct_rows(path, pb.rotated, pb.kind));
  if (waves > wmax) waves = wmax;
  return waves < 1 ? 1 : waves;
}

ShapeKey shape_key(int path, const DevProb &pb, int n) {
  ShapeKey k;
  k.path = path;
  k.dbucket = pb.D <= 16 ? 0 : pb.D <= 32 ? 1 : pb.D <= 64 ? 2 : pb.D <= 96 ? 3 : 4;
  k.fclass = 2 * pb.kind + (pb.rotated ? 1 : 0);
  int lg = 0;
  while (lg < 30 && (1 << (lg + 1)) <= n) ++lg;
  k.nbucket = lg < 4 ? 4 : (lg > 24 ? 24 : lg);
  return k;
}

void set_shape_override(const ShapeKey &k, int waves, int grid_per8) {
  overrides()[std::make_tuple(k.path, k.dbucket, k.fclass, k.nbucket)] = std::make_pair(waves, grid_per8);
}

void clear_shape_overrides() { overrides().clear(); }

void erase_shape_override(const ShapeKey &k) {
  overrides().erase(std::make_tuple(k.path, k.dbucket, k.fclass, k.nbucket));
}

bool get_shape_override(const ShapeKey &k, int *waves, int *grid_per8) {
  auto it = overrides().find(std::make_tuple(k.path, k.dbucket, k.fclass, k.nbucket));
  if (it == overrides().end()) return false;
  *waves = it->second.first;
  *grid_per8 = it->second.second;
  return true;
}

LaunchShape resident_shape_for(int path, const DevProb &pb, int n, int num_cu, int waves, int grid_per8) {
  const int wmax = resident_max_waves(path, pb);
  if (waves > wmax) waves = wmax;
  if (waves < 1) waves = 1;
  return shape_with(path, pb, n, num_cu, waves, grid_per8);
}

LaunchShape resident_shape(int path, const DevProb &pb, int n, int num_cu) {
  int ow = 0, og = 0;
  if (!overrides().empty() && get_shape_override(shape_key(path, pb, n), &ow, &og))
    return resident_shape_for(path, pb, n, num_cu, ow, og);
  int waves = resident_max_waves(path, pb);
  const int rows = kRowsPerBlock * blocks_of(path);
  const int groups = (n + rows - 1) / rows;
  // small populations: fewer waves per workgroup spread the groups over more CUs
  while (waves > 1 && (groups + waves - 1) / waves < num_cu) waves >>= 1;
  return shape_with(path, pb, n, num_cu, waves, 0);
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
