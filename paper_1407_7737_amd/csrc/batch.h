// batch.h -- batched populations (many small populations of uneven size, dimension and
// function) evaluated by one persistent launch and replayed as a HIP graph.
//
// Population i is Tab. 1 function fids[i] (with that function's transform) at dimension
// dims[i] <= 128, its random data keyed by (seed, dims[i], kBatchKeyBase + i).  Every
// population is evaluated on the FP32 split path, three or six BF16 products as the default
// mode picks per formula.  The work is cut into items of up to `groups_per_item` row groups
// (32 rows each) of one population; a host-side longest-processing-time schedule assigns
// the items to `grid` workgroups of `waves` waves.  Each workgroup walks its own item list,
// reloading the problem tables into LDS only when the population changes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "devprob.h"
#include "problem.h"

namespace curob {

constexpr uint32_t kBatchKeyBase = 2048;  // population i keys its random data by kBatchKeyBase + i
constexpr int kBatchMaxWaves = 4;
constexpr int kBatchRows = kRowsPerBlock * blocks_of(PATH_SPLIT);  // rows per row group on the FP32 paths

// The variants (formula family, rotation, six products) the batch kernel runs: one per
// Tab. 1 function fid (its family and transform, the sphere evaluated without its rotation as
// it is rotation invariant, six products where the default split mode uses them), plus
// Rosenbrock below dimension 10, which the default mode gives six products.  The elliptic
// function from dimension 50 on takes three products: the variant of id 1 (same family and
// transform kind, three products).
struct BatchVariant {
  int kind, rot, six;
};
constexpr int kBatchVariants = 24;
__host__ __device__ constexpr BatchVariant batch_variant(int v) {
  constexpr BatchVariant t[kBatchVariants] = {
      {K_WSPHERE, 0, 0},     {K_WSPHERE, 1, 0},  {K_WSPHERE, 1, 1}, {K_WSPHERE, 1, 1}, {K_WSPHERE, 1, 0},
      {K_POWERS, 1, 0},      {K_SHARPV, 1, 0},   {K_STEP, 1, 1},    {K_WEIERSTRASS, 1, 1}, {K_GRIEWANK, 1, 0},
      {K_RASTRIGIN, 0, 0},   {K_RASTRIGIN, 1, 0}, {K_F7, 1, 1},     {K_GRIEROSEN, 1, 1}, {K_ROSENBROCK, 1, 0},
      {K_SCHWEFEL, 0, 0},    {K_SCHWEFEL, 1, 1}, {K_KATSUURA, 1, 1}, {K_LUNACEK, 1, 0},  {K_ACKLEY, 1, 0},
      {K_HAPPYCAT, 1, 0},    {K_HGBAT, 1, 0},    {K_F6, 1, 0},      {K_ROSENBROCK, 1, 1}};
  return t[v];
}
inline int batch_variant_of(int fid, int dim) {
  if (fid == 14 && dim < 10) return 23;
  if (fid == 2 && dim >= 50) return 1;
  return fid;
}

// Launches the persistent batch kernel: probs/variants/xs/outs/counts per population, items
// (population, first row group, end row group, 0) and per-workgroup item ranges
// wg_begin[0..grid] in device memory.
hipError_t launch_batch(const DevProb *probs, const int *variants, const void *const *xs, void *const *outs,
                        const int *counts, const int4 *items, const int *wg_begin, int grid, int waves, int lds,
                        hipStream_t st);

}  // namespace curob
