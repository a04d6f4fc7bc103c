// composite_blend.hip -- composition functions (Sec. 6, Eqs. (composition) and (weight)):
// given the component values G_i of each row, F = sum_i omega_i (lambda_i G_i + bias_i) + f_opt
// with w_i = exp(-d_i^2 / (2 D sigma_i^2)) / d_i, d_i = |x - o^i|, omega = w / sum w.
// One wave per four rows; distances and weights in FP64 (log domain, so far rows cannot
// underflow every weight to zero); where some d_i = 0 the weights are one-hot over those
// components.
#include <hip/hip_runtime.h>

namespace curob {

// Rows per wave: each shift o^i read from memory serves kBlendRows rows, and the weights of
// the kBlendRows x 8 (row, component) pairs are computed by as many lanes at once.
constexpr int kBlendRows = 4;
constexpr int kBlendComps = 8;

template <typename T>
__global__ __launch_bounds__(256) void k_blend(const T *__restrict__ x, int n, int D, int nc, const double *__restrict__ o,
                                               const double *__restrict__ sigma, const double *__restrict__ lambda,
                                               const double *__restrict__ bias, const T *__restrict__ G, int gstride,
                                               double fopt, T *__restrict__ out) {
  constexpr int R = kBlendRows, C = kBlendComps, V = R * C;  // V = 32 (row, component) pairs
  const int lane = threadIdx.x & 63;
  const int row0 = (blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) * R;
  if (row0 >= n) return;
  // partial d_i^2 of this lane's columns: v[r * C + i] for row row0 + r, component i
  double v[V];
#pragma unroll
  for (int k = 0; k < V; ++k) v[k] = 0.0;
  // no branch around the loads (rows past n read row n - 1, components past nc the last one;
  // neither result is used), so each column step issues all its loads before the first wait
  for (int j = lane; j < D; j += 64) {
    T xr[R];
    double oi[C];
#pragma unroll
    for (int r = 0; r < R; ++r) xr[r] = x[static_cast<size_t>(row0 + r < n ? row0 + r : n - 1) * D + j];
#pragma unroll
    for (int i = 0; i < C; ++i) oi[i] = o[static_cast<size_t>(i < nc ? i : nc - 1) * D + j];
    // keep the loads together ahead of the arithmetic (the scheduler would interleave them
    // with it, one wait per load)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < C; ++i)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double d = static_cast<double>(xr[r]) - oi[i];
        v[r * C + i] += d * d;
      }
  }
  // reduce-scatter over the lanes: at each halving step a lane keeps one half of its live
  // values, adds the partner's copy of that half and hands over the other half.  After the
  // steps over lane bits 5..1, pair k = lane >> 1 is summed over 32 lanes; the step over bit 0
  // completes it in both lanes 2k and 2k + 1.
  int live = V;
#pragma unroll
  for (int m = 32; m >= 2; m >>= 1) {
    const bool up = (lane & m) != 0;
#pragma unroll
    for (int h = 0; h < V / 2; ++h) {
      if (h < live / 2) {
        const double send = up ? v[h] : v[h + live / 2];
        const double keep = up ? v[h + live / 2] : v[h];
        v[h] = keep + __shfl_xor(send, m, 64);
      }
    }
    live /= 2;
  }
  const double d2 = v[0] + __shfl_xor(v[0], 1, 64);
  // lane: row r = lane >> 4, component i = (lane >> 1) & 7; the 8 components of a row are the
  // even (or odd) lanes of its 16, combined over lane bits 1..3
  const int r = lane >> 4, i = (lane >> 1) & (C - 1);
  const int row = row0 + r;
  const bool act = i < nc;
  const bool zero = act && d2 == 0.0;
  int nzero = zero ? 1 : 0;
  double a = -1.0e308;
  if (act && !zero) a = -0.5 * log(d2) - d2 / (2.0 * D * sigma[i] * sigma[i]);
  double amax = a;
#pragma unroll
  for (int m = 2; m <= 8; m <<= 1) {
    nzero += __shfl_xor(nzero, m, 64);
    amax = fmax(amax, __shfl_xor(amax, m, 64));
  }
  double w = 0.0;
  if (act) w = nzero ? (zero ? 1.0 : 0.0) : exp(a - amax);
  double g = 0.0;
  if (act && row < n) g = w * (lambda[i] * static_cast<double>(G[static_cast<size_t>(i) * gstride + row]) + bias[i]);
  double wsum = w;
#pragma unroll
  for (int m = 2; m <= 8; m <<= 1) {
    wsum += __shfl_xor(wsum, m, 64);
    g += __shfl_xor(g, m, 64);
  }
  if ((lane & 15) == 0 && row < n) out[row] = static_cast<T>(g / wsum + fopt);
}

hipError_t launch_blend(bool f64, const void *x, int n, int D, int nc, const double *o, const double *sigma,
                        const double *lambda, const double *bias, const void *G, int gstride, double fopt, void *out,
                        hipStream_t st) {
  const dim3 grid((n + 4 * kBlendRows - 1) / (4 * kBlendRows)), block(256);
  if (f64)
    hipLaunchKernelGGL(k_blend<double>, grid, block, 0, st, static_cast<const double *>(x), n, D, nc, o, sigma, lambda,
                       bias, static_cast<const double *>(G), gstride, fopt, static_cast<double *>(out));
  else
    hipLaunchKernelGGL(k_blend<float>, grid, block, 0, st, static_cast<const float *>(x), n, D, nc, o, sigma, lambda,
                       bias, static_cast<const float *>(G), gstride, fopt, static_cast<float *>(out));
  return hipGetLastError();
}

}  // namespace curob
