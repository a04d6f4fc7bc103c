// eval_resident.hip -- fused evaluation kernel for basic functions of dimension <= 128.
//
// One wave evaluates 16 candidate rows at a time:
//   1. stage   the 16 x D block of x (contiguous in HBM) with 16-byte loads, form
//              y = s (x - o) and store it row-major in the wave's LDS slice;
//   2. rotate  Z^T = Qp Y^T on the matrix cores, tile by tile over the nonzero tiles of the
//              packed block-diagonal rotation (Sec. 1.2: three random variable groups, one
//              orthonormal block each).  The B operand is gathered from LDS in group order;
//              for the split path each y is split into bf16 hi + lo and three products
//              hi*hi + hi*lo + lo*hi accumulate in FP32;
//   3. phi     add the offset c and apply the formula to the lane's accumulator fragment
//              (pairwise families first exchange z through LDS to reach z_{i+1});
//   4. reduce  per-lane compensated sums, then a two-step cross-lane combine, finalise the
//              formula and write one value per row.
// The rotation tiles and per-position tables sit in LDS once per workgroup; each wave then
// loops over row groups (grid-stride) without further workgroup barriers.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "devprob.h"
#include "formulas.h"
#include "kernels.h"

namespace curob {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <int P>
struct PathT;
template <>
struct PathT<PATH_SPLIT> {
  using T = float;
  using V = f32x4;   // 16-byte staging vector
  using Acc4 = f32x4;
  static constexpr int KW = 32;
};
template <>
struct PathT<PATH_SPLIT6> {
  using T = float;
  using V = f32x4;
  using Acc4 = f32x4;
  static constexpr int KW = 32;
};
template <>
struct PathT<PATH_F32> {
  using T = float;
  using V = f32x4;
  using Acc4 = f32x4;
  static constexpr int KW = 4;
};
template <>
struct PathT<PATH_F64> {
  using T = double;
  using V = f64x2;
  using Acc4 = f64x4;
  static constexpr int KW = 4;
};

// Packed position held in accumulator element e of m-tile m by lane group q (= lane / 16).
// BF16 16x16x32 and FP32 16x16x4 place output row 4q+e in element e; FP64 16x16x4 places
// output row 4e+q there.
template <int P>
__device__ __forceinline__ int frag_pos(int m, int q, int e) {
  if constexpr (P == PATH_F64) return 16 * m + 4 * e + q;
  else return 16 * m + 4 * q + e;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void copy_to_lds(unsigned char *dst, const void *src, int bytes) {
  const int4 *s = reinterpret_cast<const int4 *>(src);
  int4 *d = reinterpret_cast<int4 *>(dst);
  for (int i = threadIdx.x; i < (bytes >> 4); i += blockDim.x) d[i] = s[i];
}

// Stage rows [row0, row0 + nrows) of x into Y (row stride S): Y[r][j] = s_j (x[r][j] - o_j).
// FP32 paths subtract o as a hi + lo pair: x - o_hi is exact near the optimum, so y keeps
// its relative accuracy where the formula weights (up to 1e6) would amplify an absolute error.
template <int P>
__device__ __forceinline__ void stage(const typename PathT<P>::T *__restrict__ xg, int tot, int D, int S, bool vec,
                                      typename PathT<P>::T *Y, const typename PathT<P>::T *so,
                                      const typename PathT<P>::T *sol, const typename PathT<P>::T *ss, int lane) {
  using T = typename PathT<P>::T;
  using V = typename PathT<P>::V;
  constexpr int NV = 16 / sizeof(T);
  if (vec) {
    // 16 rows x at most 128 elements, NV elements per load
    constexpr int TMAX = (kRowsPerWave * 128) / (64 * NV);
    V v[TMAX];
#pragma unroll
    for (int t = 0; t < TMAX; ++t) {
      const int e = (lane + 64 * t) * NV;
      if (e < tot) v[t] = *reinterpret_cast<const V *>(xg + e);
    }
    const int e0 = lane * NV;
    int rr = e0 / D, jj = e0 - rr * D;
    const int step = 64 * NV;
    const int dr = step / D, dj = step - dr * D;
#pragma unroll
    for (int t = 0; t < TMAX; ++t) {
      const int e = (lane + 64 * t) * NV;
      if (e < tot) {
        const V ov = *reinterpret_cast<const V *>(so + jj);
        const V sv = *reinterpret_cast<const V *>(ss + jj);
        V d = v[t] - ov;
        if constexpr (P != PATH_F64) d -= *reinterpret_cast<const V *>(sol + jj);
        *reinterpret_cast<V *>(Y + rr * S + jj) = sv * d;
      }
      jj += dj;
      rr += dr;
      if (jj >= D) {
        jj -= D;
        ++rr;
      }
    }
  } else {
    constexpr int TMAX = (kRowsPerWave * 128) / 64;
    T v[TMAX];
#pragma unroll
    for (int t = 0; t < TMAX; ++t) {
      const int e = lane + 64 * t;
      if (e < tot) v[t] = xg[e];
    }
    int rr = lane / D, jj = lane - rr * D;
    const int dr = 64 / D, dj = 64 - dr * D;
#pragma unroll
    for (int t = 0; t < TMAX; ++t) {
      const int e = lane + 64 * t;
      if (e < tot) {
        T d = v[t] - so[jj];
        if constexpr (P != PATH_F64) d -= sol[jj];
        Y[rr * S + jj] = ss[jj] * d;
      }
      jj += dj;
      rr += dr;
      if (jj >= D) {
        jj -= D;
        ++rr;
      }
    }
  }
}

// Z^T = Qp Y^T for the wave's 16 rows; z[m][e] receives packed position frag_pos(m, q, e).
template <int P>
__device__ __forceinline__ void rotate(typename PathT<P>::T (&z)[kMaxMT][4], const DevProb &pb,
                                       const unsigned char *s_q, const uint16_t *s_orig,
                                       const typename PathT<P>::T *Y, int r, int q, int lane) {
  using T = typename PathT<P>::T;
  using Acc4 = typename PathT<P>::Acc4;
  Acc4 acc[kMaxMT];
#pragma unroll
  for (int m = 0; m < kMaxMT; ++m) acc[m] = Acc4{0, 0, 0, 0};
  const T *Yr = Y + r * pb.S;
  const int4 *ktab = reinterpret_cast<const int4 *>(pb.ktab);
  for (int kt = 0; kt < pb.KT; ++kt) {
    const int4 ki = ktab[kt];  // uniform: scalar load
    if constexpr (P == PATH_SPLIT || P == PATH_SPLIT6) {
      // this lane's 8 inputs: packed positions 32 kt + 8 q + 0..7, split into bf16 terms
      // (y - hi and the next residual are exact in FP32)
      const uint4 idx = *reinterpret_cast<const uint4 *>(s_orig + kt * 32 + q * 8);
      const uint32_t iw[4] = {idx.x, idx.y, idx.z, idx.w};
      bf16x8 bh, bm, bl;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const uint32_t j = (iw[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
        const float y = Yr[j];
        const __bf16 h = (__bf16)y;
        const float r1 = y - (float)h;
        bh[e] = h;
        if constexpr (P == PATH_SPLIT6) {
          const __bf16 mm = (__bf16)r1;
          bm[e] = mm;
          bl[e] = (__bf16)(r1 - (float)mm);
        } else {
          bl[e] = (__bf16)r1;
        }
      }
      const bf16x8 *qf = reinterpret_cast<const bf16x8 *>(s_q);
#pragma unroll
      for (int m = 0; m < kMaxMT; ++m) {
        if (m >= ki.x && m <= ki.y) {
          const int t = ki.z + m - ki.x;
          if constexpr (P == PATH_SPLIT6) {
            // keep the six products of total order <= 2 in the 2^-8 splitting, smallest first
            const bf16x8 ah = qf[t * 192 + lane];
            const bf16x8 am = qf[t * 192 + 64 + lane];
            const bf16x8 al = qf[t * 192 + 128 + lane];
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[m], 0, 0, 0);
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm, acc[m], 0, 0, 0);
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[m], 0, 0, 0);
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh, acc[m], 0, 0, 0);
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm, acc[m], 0, 0, 0);
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[m], 0, 0, 0);
          } else {
            const bf16x8 ah = qf[t * 128 + lane];
            const bf16x8 al = qf[t * 128 + 64 + lane];
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[m], 0, 0, 0);
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[m], 0, 0, 0);
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[m], 0, 0, 0);
          }
        }
      }
    } else {
      const T b = Yr[s_orig[kt * 4 + q]];
      const T *qf = reinterpret_cast<const T *>(s_q);
#pragma unroll
      for (int m = 0; m < kMaxMT; ++m) {
        if (m >= ki.x && m <= ki.y) {
          const T a = qf[(ki.z + m - ki.x) * 64 + lane];
          if constexpr (P == PATH_F64)
            acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[m], 0, 0, 0);
          else
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[m], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int m = 0; m < kMaxMT; ++m)
#pragma unroll
    for (int e = 0; e < 4; ++e) z[m][e] = acc[m][e];
}

template <int P, int KIND>
__global__ __launch_bounds__(256) void k_eval_resident(DevProb pb, const typename PathT<P>::T *__restrict__ x,
                                                       typename PathT<P>::T *__restrict__ out, int n, int vec) {
  using T = typename PathT<P>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  const LdsLayout L = lds_layout(P, pb);
  unsigned char *s_q = smem + L.q;
  T *s_o = reinterpret_cast<T *>(smem + L.o);
  T *s_ol = reinterpret_cast<T *>(smem + L.olo);
  T *s_s = reinterpret_cast<T *>(smem + L.s);
  uint16_t *s_orig = reinterpret_cast<uint16_t *>(smem + L.orig);
  T *s_coef = reinterpret_cast<T *>(smem + L.coef);
  T *s_cz = reinterpret_cast<T *>(smem + L.cz);
  int16_t *s_succ = reinterpret_cast<int16_t *>(smem + L.succ);
  T *s_y = reinterpret_cast<T *>(smem + L.y);

  if (pb.rotated) {
    copy_to_lds(s_q, pb.qfrag, L.q_bytes);
    copy_to_lds(reinterpret_cast<unsigned char *>(s_orig), pb.orig, L.orig_bytes);
  }
  copy_to_lds(reinterpret_cast<unsigned char *>(s_o), pb.o, L.vec_bytes);
  if (P != PATH_F64) copy_to_lds(reinterpret_cast<unsigned char *>(s_ol), pb.olo, L.vec_bytes);
  copy_to_lds(reinterpret_cast<unsigned char *>(s_s), pb.sj, L.vec_bytes);
  copy_to_lds(reinterpret_cast<unsigned char *>(s_coef), pb.coef, L.mp_bytes);
  copy_to_lds(reinterpret_cast<unsigned char *>(s_cz), pb.cz, L.mp_bytes);
  if (KindTraits<KIND>::pairwise) copy_to_lds(reinterpret_cast<unsigned char *>(s_succ), pb.succ, L.succ_bytes);
  __syncthreads();

  const int D = pb.D, S = pb.S, MT = pb.MT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  T *Y = s_y + wave * kRowsPerWave * S;
  if (lane < kRowsPerWave) Y[lane * S + D] = T(0);  // padding slot read by the gather
  const T prm = kind_param<KIND, T>(pb.Df, pb.kparam);

  const int ngroups = (n + kRowsPerWave - 1) / kRowsPerWave;
  for (int g = blockIdx.x * kWavesPerWG + wave; g < ngroups; g += gridDim.x * kWavesPerWG) {
    const int row0 = g * kRowsPerWave;
    const int nrows = min(kRowsPerWave, n - row0);
    wave_sync();
    stage<P>(x + static_cast<size_t>(row0) * D, nrows * D, D, S, vec != 0, Y, s_o, s_ol, s_s, lane);
    wave_sync();

    T z[kMaxMT][4];
    if (pb.rotated) {
      rotate<P>(z, pb, s_q, s_orig, Y, r, q, lane);
    } else {
#pragma unroll
      for (int m = 0; m < kMaxMT; ++m)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int p = frag_pos<P>(m, q, e);
          z[m][e] = (m < MT && p < D) ? Y[r * S + p] : T(0);
        }
    }
#pragma unroll
    for (int m = 0; m < kMaxMT; ++m)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int p = frag_pos<P>(m, q, e);
        if (m < MT) z[m][e] += s_cz[p];
      }

    Acc<T> a;
    a.init();
    if constexpr (KindTraits<KIND>::pairwise) {
      wave_sync();
#pragma unroll
      for (int m = 0; m < kMaxMT; ++m)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int p = frag_pos<P>(m, q, e);
          if (m < MT && p < D) Y[r * S + p] = z[m][e];
        }
      wave_sync();
#pragma unroll
      for (int m = 0; m < kMaxMT; ++m)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int p = frag_pos<P>(m, q, e);
          if (m < MT && p < D) {
            const int sp = s_succ[p];
            if (sp >= 0) phi<KIND, T>(a, z[m][e], Y[r * S + sp], T(0), prm);
          }
        }
    } else {
#pragma unroll
      for (int m = 0; m < kMaxMT; ++m)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int p = frag_pos<P>(m, q, e);
          if (m < MT && p < D) {
            const T cf = KindTraits<KIND>::needs_coef ? s_coef[p] : T(0);
            phi<KIND, T>(a, z[m][e], T(0), cf, prm);
          }
        }
    }

    // combine the four lanes that hold the same row (lane, lane^16, lane^32, lane^48)
#pragma unroll
    for (int sh = 16; sh <= 32; sh <<= 1) {
      T s[3], c[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        s[k] = __shfl_xor(a.s[k], sh, 64);
        c[k] = __shfl_xor(a.c[k], sh, 64);
      }
      const T p = __shfl_xor(a.p, sh, 64);
      acc_merge(a, s, c, p);
    }
    if (q == 0 && r < nrows) out[row0 + r] = finalize<KIND, T>(a, pb.Df) + T(pb.bias);
  }
}

// ---- launch table ----------------------------------------------------------------------

template <int P, int... Ks>
static const void *const *kernel_table(std::integer_sequence<int, Ks...>) {
  static const void *const tab[] = {reinterpret_cast<const void *>(&k_eval_resident<P, Ks>)...};
  return tab;
}

static const void *resident_kernel(int path, int kind) {
  if (kind < 0 || kind >= K_COUNT) return nullptr;
  auto seq = std::make_integer_sequence<int, K_COUNT>{};
  switch (path) {
    case PATH_SPLIT: return kernel_table<PATH_SPLIT>(seq)[kind];
    case PATH_F32: return kernel_table<PATH_F32>(seq)[kind];
    case PATH_F64: return kernel_table<PATH_F64>(seq)[kind];
    case PATH_SPLIT6: return kernel_table<PATH_SPLIT6>(seq)[kind];
    default: return nullptr;
  }
}

int resident_grid(int path, const DevProb &pb, int n, int num_cu) {
  const LdsLayout L = lds_layout(path, pb);
  const void *fn = resident_kernel(path, pb.kind);
  int occ = 0;
  if (fn == nullptr ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, 64 * kWavesPerWG, static_cast<size_t>(L.total)) !=
          hipSuccess)
    occ = 1;
  if (occ < 1) occ = 1;
  const int groups = (n + kRowsPerWave - 1) / kRowsPerWave;
  const int need = (groups + kWavesPerWG - 1) / kWavesPerWG;
  const int cap = occ * num_cu;
  return need < cap ? (need > 0 ? need : 1) : cap;
}

hipError_t launch_resident(int path, const DevProb &pb, const void *x, void *out, int n, int grid, hipStream_t st) {
  const void *fn = resident_kernel(path, pb.kind);
  if (fn == nullptr) return hipErrorInvalidValue;
  const LdsLayout L = lds_layout(path, pb);
  if (L.total > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, L.total);
    if (e != hipSuccess) return e;
  }
  const size_t esz = path == PATH_F64 ? 8 : 4;
  int vec = ((pb.D % static_cast<int>(16 / esz)) == 0 && (reinterpret_cast<uintptr_t>(x) % 16) == 0) ? 1 : 0;
  DevProb arg = pb;
  const void *xa = x;
  void *oa = out;
  void *args[] = {&arg, &xa, &oa, &n, &vec};
  return hipLaunchKernel(fn, dim3(grid), dim3(64 * kWavesPerWG), args, static_cast<size_t>(L.total), st);
}

}  // namespace curob
