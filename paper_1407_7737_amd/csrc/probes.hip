// probes.hip -- measured peaks for the roofline: the streaming read bandwidth of device
// memory and the dense BF16 matrix-core rate, each on a full-occupancy grid, timed with HIP
// events on the library stream.  They evaluate nothing; a benchmark reports them beside the
// nominal peaks.
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/curob.h"

namespace curob {
hipStream_t context_stream();
bool context_ready();
int context_num_cu();
int set_error(int code, const std::string &msg);
}  // namespace curob

using namespace curob;

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;

// Every 16-byte word of [buf, buf + words) is loaded once (grid-stride, four loads in flight
// per thread) and folded into one value per thread; a thread stores only if its fold has an
// impossible pattern, so the kernel writes no memory in practice.
__global__ __launch_bounds__(256) void k_probe_read(const u32x4 *__restrict__ buf, unsigned long long words,
                                                    unsigned *__restrict__ sink) {
  const unsigned long long stride = static_cast<unsigned long long>(gridDim.x) * blockDim.x;
  unsigned long long i = static_cast<unsigned long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  u32x4 a = u32x4{0u, 0u, 0u, 0u}, b = a, c = a, d = a;
  for (; i + 3 * stride < words; i += 4 * stride) {
    a ^= buf[i];
    b ^= buf[i + stride];
    c ^= buf[i + 2 * stride];
    d ^= buf[i + 3 * stride];
  }
  for (; i < words; i += stride) a ^= buf[i];
  const u32x4 v = a ^ b ^ c ^ d;
  if ((v.x & v.y & v.z & v.w) == 0xFFFFFFFFu) sink[0] = v.x;
}

// Each wave runs `iters` rounds of four independent accumulation chains of 16x16x32 BF16
// MFMAs (operands fixed, so the matrix cores do nothing else); a lane stores only if its
// result has an impossible value.
constexpr int kProbeChains = 4;
__global__ __launch_bounds__(256) void k_probe_mfma(int iters, float *__restrict__ sink) {
  bf16x8 a, b;
  for (int e = 0; e < 8; ++e) {
    a[e] = static_cast<__bf16>(0.001f * static_cast<float>((threadIdx.x + e) & 15));
    b[e] = static_cast<__bf16>(0.002f * static_cast<float>(e));
  }
  f32x4 c0 = f32x4{0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
  for (int i = 0; i < iters; ++i) {
    c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c3, 0, 0, 0);
  }
  const f32x4 s = c0 + c1 + c2 + c3;
  if (s[0] == -1.0f) sink[0] = s[1];
}

// Fastest of `reps` launches of fn on the library stream, in milliseconds.
template <typename F>
int best_ms(F launch, int reps, float *ms, const char *what) {
  hipStream_t st = context_stream();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  if (he == hipSuccess) he = launch(st);  // warm-up
  float best = -1.0f;
  for (int r = 0; r < reps && he == hipSuccess; ++r) {
    he = hipEventRecord(e0, st);
    if (he == hipSuccess) he = launch(st);
    if (he == hipSuccess) he = hipEventRecord(e1, st);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float t = 0.0f;
    if (he == hipSuccess) he = hipEventElapsedTime(&t, e0, e1);
    if (he == hipSuccess && (best < 0.0f || t < best)) best = t;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (he != hipSuccess) return set_error(CUROB_E_HIP, std::string(what) + ": " + hipGetErrorString(he));
  *ms = best;
  return CUROB_OK;
}

}  // namespace

extern "C" int curob_probe_read(const void *d_buf, unsigned long long bytes, int reps, double *gbs) {
  if (!context_ready()) return set_error(CUROB_E_STATE, "curob_probe_read: library not initialised");
  if (d_buf == nullptr || gbs == nullptr || bytes < 16 || bytes % 16 != 0 || reps < 1 ||
      reinterpret_cast<uintptr_t>(d_buf) % 16 != 0)
    return set_error(CUROB_E_ARG, "curob_probe_read: need a 16-byte aligned device buffer of a positive multiple "
                                  "of 16 bytes, reps >= 1 and an output pointer");
  unsigned *sink = nullptr;
  hipError_t he = hipMalloc(&sink, 16);
  if (he != hipSuccess) return set_error(CUROB_E_HIP, std::string("curob_probe_read: ") + hipGetErrorString(he));
  const unsigned long long words = bytes / 16;
  const int grid = 8 * context_num_cu();
  const u32x4 *buf = static_cast<const u32x4 *>(d_buf);
  float ms = 0.0f;
  int rc = best_ms(
      [&](hipStream_t st) {
        hipLaunchKernelGGL(k_probe_read, dim3(grid), dim3(256), 0, st, buf, words, sink);
        return hipGetLastError();
      },
      reps, &ms, "curob_probe_read");
  (void)hipFree(sink);
  if (rc != CUROB_OK) return rc;
  *gbs = static_cast<double>(bytes) / (static_cast<double>(ms) * 1e-3) / 1e9;
  return CUROB_OK;
}

extern "C" int curob_probe_mfma_bf16(int reps, double *tflops) {
  if (!context_ready()) return set_error(CUROB_E_STATE, "curob_probe_mfma_bf16: library not initialised");
  if (tflops == nullptr || reps < 1) return set_error(CUROB_E_ARG, "curob_probe_mfma_bf16: reps >= 1 and an output pointer");
  float *sink = nullptr;
  hipError_t he = hipMalloc(&sink, 16);
  if (he != hipSuccess) return set_error(CUROB_E_HIP, std::string("curob_probe_mfma_bf16: ") + hipGetErrorString(he));
  // four 4-wave workgroups per CU: four waves per SIMD
  const int grid = 4 * context_num_cu(), iters = 4096;
  float ms = 0.0f;
  int rc = best_ms(
      [&](hipStream_t st) {
        hipLaunchKernelGGL(k_probe_mfma, dim3(grid), dim3(256), 0, st, iters, sink);
        return hipGetLastError();
      },
      reps, &ms, "curob_probe_mfma_bf16");
  (void)hipFree(sink);
  if (rc != CUROB_OK) return rc;
  const double mfmas = static_cast<double>(grid) * 4.0 * iters * kProbeChains;
  *tflops = mfmas * 2.0 * 16 * 16 * 32 / (static_cast<double>(ms) * 1e-3) / 1e12;
  return CUROB_OK;
}
