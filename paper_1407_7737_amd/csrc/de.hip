// de.hip -- differential evolution (DE/rand/1/bin) around the evaluation calls: the paper's
// motivating use (Sec. 1: optimisation algorithms running on the GPU call the benchmark's
// evaluation interface directly; Sec. 2: 50 concurrent evaluations per call).
//
// One generation = trial vectors (k_de_trial), their evaluation through func_evaluate[f], and
// greedy selection (k_de_select), all enqueued on one stream with no allocation, copy or
// memset, so any number of generations can be captured in one HIP graph.  The generation
// counter lives in device memory and k_de_select advances it, so replaying a captured graph
// continues the sequence instead of repeating it.
//
// Random numbers are counter based: draw k of a run is the published SplitMix64 output for
// state seed + (k + 1) * 0x9E3779B97F4A7C15 (Steele, Lea & Flood 2014), k = ((g * np + i) *
// (D + 4)) + slot for individual i of generation g; slots 0-2 choose r1, r2, r3, slot 3 the
// forced crossover position, slot 4 + j the crossover draw of variable j.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace curob {

namespace {

__device__ __forceinline__ uint64_t de_draw(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// An index in 0..np-1 outside the m (<= 3) distinct excluded ones: the draw picks the v-th
// (0-based) of the np - m allowed values in increasing order.
__device__ __forceinline__ int de_pick(uint64_t u, int np, const int *ex, int m) {
  int v = static_cast<int>(u % static_cast<uint64_t>(np - m));
  // excluded values in increasing order
  int e[3] = {ex[0], m > 1 ? ex[1] : 0x7fffffff, m > 2 ? ex[2] : 0x7fffffff};
  if (e[0] > e[1]) { const int t = e[0]; e[0] = e[1]; e[1] = t; }
  if (e[1] > e[2]) { const int t = e[1]; e[1] = e[2]; e[2] = t; }
  if (e[0] > e[1]) { const int t = e[0]; e[0] = e[1]; e[1] = t; }
  for (int a = 0; a < m; ++a) v += v >= e[a] ? 1 : 0;
  return v;
}

template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c) {
  if constexpr (sizeof(T) == 4) return __builtin_fmaf(a, b, c); else return __builtin_fma(a, b, c);
}

// One wave per individual, lanes over the variables.
template <typename T>
__global__ __launch_bounds__(256) void k_de_trial(const T *__restrict__ pop, T *__restrict__ trial, int np, int D,
                                                  double F, double CR, uint64_t seed,
                                                  const unsigned long long *__restrict__ gen) {
  const int i = blockIdx.x * 4 + static_cast<int>(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= np) return;
  const uint64_t base = (static_cast<uint64_t>(gen[0]) * np + i) * static_cast<uint64_t>(D + 4);
  int ex[3] = {i, 0, 0};
  const int r1 = de_pick(de_draw(seed, base + 0), np, ex, 1);
  ex[1] = r1;
  const int r2 = de_pick(de_draw(seed, base + 1), np, ex, 2);
  ex[2] = r2;
  const int r3 = de_pick(de_draw(seed, base + 2), np, ex, 3);
  const int jr = static_cast<int>(de_draw(seed, base + 3) % static_cast<uint64_t>(D));
  const T f = static_cast<T>(F);
  for (int j = lane; j < D; j += 64) {
    const double u = static_cast<double>(de_draw(seed, base + 4 + j) >> 11) * 0x1.0p-53;
    const T xi = pop[static_cast<size_t>(i) * D + j];
    T t = xi;
    if (u < CR || j == jr) {
      const T a = pop[static_cast<size_t>(r1) * D + j];
      const T b = pop[static_cast<size_t>(r2) * D + j];
      const T c = pop[static_cast<size_t>(r3) * D + j];
      t = fma_t(f, b - c, a);
      t = t < T(-100) ? T(-100) : (t > T(100) ? T(100) : t);  // back into the search box
    }
    trial[static_cast<size_t>(i) * D + j] = t;
  }
}

// Greedy selection: a trial replaces its target when its value is not larger.  Thread 0 of
// workgroup 0 then advances the generation counter (the next generation's kernels run after
// this one on the stream).
template <typename T>
__global__ __launch_bounds__(256) void k_de_select(T *__restrict__ pop, T *__restrict__ fit,
                                                   const T *__restrict__ trial, const T *__restrict__ ftrial, int np,
                                                   int D, unsigned long long *__restrict__ gen) {
  const int i = blockIdx.x * 4 + static_cast<int>(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (blockIdx.x == 0 && threadIdx.x == 0) gen[0] = gen[0] + 1ULL;
  if (i >= np) return;
  const T ft = ftrial[i];
  if (!(ft <= fit[i])) return;
  for (int j = lane; j < D; j += 64) pop[static_cast<size_t>(i) * D + j] = trial[static_cast<size_t>(i) * D + j];
  if (lane == 0) fit[i] = ft;
}

}  // namespace

hipError_t launch_de_trial(bool f64, const void *pop, void *trial, int np, int D, double F, double CR, uint64_t seed,
                           const unsigned long long *gen, hipStream_t st) {
  const dim3 grid((np + 3) / 4), block(256);
  if (f64)
    hipLaunchKernelGGL(k_de_trial<double>, grid, block, 0, st, static_cast<const double *>(pop),
                       static_cast<double *>(trial), np, D, F, CR, seed, gen);
  else
    hipLaunchKernelGGL(k_de_trial<float>, grid, block, 0, st, static_cast<const float *>(pop),
                       static_cast<float *>(trial), np, D, F, CR, seed, gen);
  return hipGetLastError();
}

hipError_t launch_de_select(bool f64, void *pop, void *fit, const void *trial, const void *ftrial, int np, int D,
                            unsigned long long *gen, hipStream_t st) {
  const dim3 grid((np + 3) / 4), block(256);
  if (f64)
    hipLaunchKernelGGL(k_de_select<double>, grid, block, 0, st, static_cast<double *>(pop), static_cast<double *>(fit),
                       static_cast<const double *>(trial), static_cast<const double *>(ftrial), np, D, gen);
  else
    hipLaunchKernelGGL(k_de_select<float>, grid, block, 0, st, static_cast<float *>(pop), static_cast<float *>(fit),
                       static_cast<const float *>(trial), static_cast<const float *>(ftrial), np, D, gen);
  return hipGetLastError();
}

}  // namespace curob
