// eval_batch.hip -- the persistent batch kernel: each workgroup walks its item list and
// evaluates each item's row groups with the resident kernel's body for that population's
// formula variant.
#include <utility>

#include "batch.h"
#include "eval_resident.h"

namespace curob {

namespace {

template <int V>
__device__ __forceinline__ void batch_item(const DevProb &pb, const float *x, float *out, int n, int g0, int g1,
                                           int nwaves, int wave, bool setup, unsigned char *smem) {
  constexpr BatchVariant v = batch_variant(V);
  constexpr int P = v.six ? PATH_SPLIT6 : PATH_SPLIT;
  resident_eval<P, v.kind, v.rot, 0>(pb, x, out, n, g0 + wave, g1, nwaves, nwaves, wave, setup, smem);
}

template <int... Fs>
__device__ __forceinline__ void dispatch(int var, const DevProb &pb, const float *x, float *out, int n, int g0, int g1,
                                         int nwaves, int wave, bool setup, unsigned char *smem,
                                         std::integer_sequence<int, Fs...>) {
  // one wave-uniform branch per variant
  ((var == Fs ? (batch_item<Fs>(pb, x, out, n, g0, g1, nwaves, wave, setup, smem), 0) : 0), ...);
}

__global__ __launch_bounds__(64 * kBatchMaxWaves) void k_eval_batch(const DevProb *__restrict__ probs,
                                                                    const int *__restrict__ variants,
                                                                    const void *const *__restrict__ xs,
                                                                    void *const *__restrict__ outs,
                                                                    const int *__restrict__ counts,
                                                                    const int4 *__restrict__ items,
                                                                    const int *__restrict__ wg_begin) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nwaves = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int i0 = __builtin_amdgcn_readfirstlane(wg_begin[blockIdx.x]);
  const int i1 = __builtin_amdgcn_readfirstlane(wg_begin[blockIdx.x + 1]);
  int cur = -1;
  for (int it = i0; it < i1; ++it) {
    const int4 item = items[it];
    const int pop = __builtin_amdgcn_readfirstlane(item.x);
    const int g0 = __builtin_amdgcn_readfirstlane(item.y);
    const int g1 = __builtin_amdgcn_readfirstlane(item.z);
    const bool setup = pop != cur;
    if (setup) __syncthreads();  // every wave is done with the previous population's tables
    cur = pop;
    const DevProb pb = probs[pop];
    const int var = __builtin_amdgcn_readfirstlane(variants[pop]);
    const int n = __builtin_amdgcn_readfirstlane(counts[pop]);
    dispatch(var, pb, static_cast<const float *>(xs[pop]), static_cast<float *>(outs[pop]), n, g0, g1, nwaves, wave,
             setup, smem, std::make_integer_sequence<int, kBatchVariants>{});
  }
}

}  // namespace

hipError_t launch_batch(const DevProb *probs, const int *variants, const void *const *xs, void *const *outs,
                        const int *counts, const int4 *items, const int *wg_begin, int grid, int waves, int lds,
                        hipStream_t st) {
  if (waves < 1 || waves > kBatchMaxWaves || grid < 1) return hipErrorInvalidValue;
  const void *fn = reinterpret_cast<const void *>(&k_eval_batch);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
  }
  void *args[] = {&probs, &variants, &xs, &outs, &counts, &items, &wg_begin};
  return hipLaunchKernel(fn, dim3(grid), dim3(64 * waves), args, static_cast<size_t>(lds), st);
}

}  // namespace curob
