// composite_blend.hip -- composition functions (Sec. 6, Eqs. (composition) and (weight)):
// given the component values G_i of each row, F = sum_i omega_i (lambda_i G_i + bias_i) + f_opt
// with w_i = exp(-d_i^2 / (2 D sigma_i^2)) / d_i, d_i = |x - o^i|, omega = w / sum w.
// One wave per row; distances and weights in FP64 (log domain, so far rows cannot underflow
// every weight to zero); where some d_i = 0 the weights are one-hot over those components.
#include <hip/hip_runtime.h>

namespace curob {

template <typename T>
__global__ __launch_bounds__(256) void k_blend(const T *__restrict__ x, int n, int D, int nc, const double *__restrict__ o,
                                               const double *__restrict__ sigma, const double *__restrict__ lambda,
                                               const double *__restrict__ bias, const T *__restrict__ G, int gstride,
                                               double fopt, T *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (row >= n) return;
  const T *xr = x + static_cast<size_t>(row) * D;
  double d2[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) d2[i] = 0.0;
  for (int j = lane; j < D; j += 64) {
    const double xv = static_cast<double>(xr[j]);
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (i < nc) {
        const double d = xv - o[static_cast<size_t>(i) * D + j];
        d2[i] += d * d;
      }
  }
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int sh = 1; sh < 64; sh <<= 1) d2[i] += __shfl_xor(d2[i], sh, 64);
  if (lane != 0) return;
  double a[8], amax = -1.0e308;
  int nzero = 0;
  for (int i = 0; i < nc; ++i) nzero += d2[i] == 0.0;
  for (int i = 0; i < nc; ++i) {
    a[i] = d2[i] == 0.0 ? 0.0 : -0.5 * log(d2[i]) - d2[i] / (2.0 * D * sigma[i] * sigma[i]);
    if (nzero == 0 && a[i] > amax) amax = a[i];
  }
  double wsum = 0.0, F = 0.0;
  for (int i = 0; i < nc; ++i) {
    const double w = nzero ? (d2[i] == 0.0 ? 1.0 : 0.0) : exp(a[i] - amax);
    wsum += w;
    F += w * (lambda[i] * static_cast<double>(G[static_cast<size_t>(i) * gstride + row]) + bias[i]);
  }
  out[row] = static_cast<T>(F / wsum + fopt);
}

hipError_t launch_blend(bool f64, const void *x, int n, int D, int nc, const double *o, const double *sigma,
                        const double *lambda, const double *bias, const void *G, int gstride, double fopt, void *out,
                        hipStream_t st) {
  const dim3 grid((n + 3) / 4), block(256);
  if (f64)
    hipLaunchKernelGGL(k_blend<double>, grid, block, 0, st, static_cast<const double *>(x), n, D, nc, o, sigma, lambda,
                       bias, static_cast<const double *>(G), gstride, fopt, static_cast<double *>(out));
  else
    hipLaunchKernelGGL(k_blend<float>, grid, block, 0, st, static_cast<const float *>(x), n, D, nc, o, sigma, lambda,
                       bias, static_cast<const float *>(G), gstride, fopt, static_cast<float *>(out));
  return hipGetLastError();
}

}  // namespace curob
