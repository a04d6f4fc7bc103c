// kernels.h -- launch entry points of the evaluation kernels and the LDS layout they share
// with the host-side table builder.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "devprob.h"
#include "problem.h"

namespace curob {

struct LdsLayout {
  int q, goff, oh, cz, coef, succ, mtab, y;  // byte offsets
  int q_bytes, goff_bytes, vec_bytes, mp_bytes, succ_bytes, mtab_bytes, slice_bytes;
  int fixed;  // bytes before the per-wave slices
  int total;
};

__host__ __device__ inline int round16(int b) { return (b + 15) & ~15; }

constexpr int kMaxLdsBytes = 160 * 1024;  // LDS per workgroup on gfx950

// Rotated problems on the split paths whose formula reads no successor take their rows from
// memory straight into the wave's LDS slice (buffer loads that write LDS): no registers hold the
// rows on the way, and the slice needs no spill row.  The pairwise families write z back into
// the slice, so they stage through registers.
__host__ __device__ constexpr bool direct_rows(int path, int rotated, int kind) {
  return is_split(path) && rotated != 0 && kind != K_F7 && kind != K_GRIEROSEN && kind != K_ROSENBROCK &&
         kind != K_F6;
}

// Waves per workgroup of the resident kernel: one 16-row column block per wave, so the per-wave
// LDS slice is small and up to four waves share a SIMD (<= 128 VGPRs) on the split paths; the
// six-product path holds a third B term, so with rows staged through registers it keeps three
// waves per SIMD (<= 168 VGPRs).  The FP64 path is bound by LDS to about eight waves.
__host__ __device__ constexpr int max_waves_of(int path, bool direct) {
  return path == PATH_F64 ? 8 : (path == PATH_SPLIT6 && !direct ? 12 : 16);
}

// LDS carve of the resident kernel: rotation tiles, gather offsets, per-variable shift,
// per-position tables, the per-m-tile k ranges, then one slice per wave holding its rows (16 per
// column block) plus, when the rows are staged through registers, one spill row, S elements each.
__host__ __device__ inline LdsLayout lds_layout(int path, const DevProb &pb, int nwaves) {
  const int esz = path == PATH_F64 ? 8 : 4;
  const int kw = kw_of(path);
  const int rows = kRowsPerBlock * blocks_of(path);
  LdsLayout L;
  L.q_bytes = pb.rotated ? round16(pb.ntiles * 64 * (is_split(path) ? 16 * split_terms(path) : esz)) : 0;
  L.goff_bytes = pb.rotated ? round16(pb.KT * kw * 2) : 0;
  // o_hi: original order (D entries), or packed order on the split paths (KT * KW and 16 * MT
  // positions, zeros past D)
  const int nvec = is_split(path) ? (pb.KT * kw > 16 * pb.MT ? pb.KT * kw : 16 * pb.MT) : pb.D;
  L.vec_bytes = round16((nvec > pb.D ? nvec : pb.D) * esz);
  L.mp_bytes = round16(16 * pb.MT * esz);
  L.succ_bytes = round16(16 * pb.MT * 2);
  L.mtab_bytes = pb.rotated ? 16 * pb.MT : 0;
  L.slice_bytes = round16((rows + (direct_rows(path, pb.rotated, pb.kind) ? 0 : 1)) * pb.S * esz);
  int off = 0;
  L.q = off;
  off += L.q_bytes;
  L.goff = off;
  off += L.goff_bytes;
  L.oh = off;
  off += L.vec_bytes;
  L.cz = off;
  off += L.mp_bytes;
  L.coef = off;
  off += L.mp_bytes;
  L.succ = off;
  off += L.succ_bytes;
  L.mtab = off;
  off += L.mtab_bytes;
  L.y = off;
  L.fixed = off;
  off += L.slice_bytes * nwaves;
  L.total = off;
  return L;
}

// Launch shape of the resident kernel for one problem: waves per workgroup (as many as the
// LDS slices allow, up to 8) and a persistent grid of at most `occupancy x CUs` workgroups.
struct LaunchShape {
  int waves;
  int grid;
  int lds;
};
LaunchShape resident_shape(int path, const DevProb &pb, int n, int num_cu);

// Autotuned launch shapes.  A key is (path, D bucket, formula class, row-count bucket): D
// buckets 0..4 for D <= 16, 32, 64, 96, 128; the class is 2 * kind + rotated; the row bucket is
// floor(log2 n) clamped to 4..24.  An entry fixes the waves per workgroup and the workgroups
// per 8 CUs of the resident kernel (clamped to what the LDS and the occupancy allow).
struct ShapeKey {
  int path, dbucket, fclass, nbucket;
};
ShapeKey shape_key(int path, const DevProb &pb, int n);
void set_shape_override(const ShapeKey &k, int waves, int grid_per8);
void clear_shape_overrides();
void erase_shape_override(const ShapeKey &k);
bool get_shape_override(const ShapeKey &k, int *waves, int *grid_per8);
// Largest waves per workgroup the LDS and the path allow for this problem.
int resident_max_waves(int path, const DevProb &pb);
// The shape for an explicit (waves, workgroups per 8 CUs), clamped like an override.
LaunchShape resident_shape_for(int path, const DevProb &pb, int n, int num_cu, int waves, int grid_per8);

// Resident kernel (dimension <= 128): evaluates n rows of x (device, row-major) into out.
hipError_t launch_resident(int path, const DevProb &pb, const void *x, void *out, int n, const LaunchShape &ls,
                           hipStream_t st);

}  // namespace curob
