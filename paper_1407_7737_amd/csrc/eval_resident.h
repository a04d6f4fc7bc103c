// eval_resident.h -- fused evaluation kernel for basic functions of dimension <= 128.
//
// Each wave evaluates 16 candidate rows at a time and loops over row groups (grid-stride):
//   1. stage   the 16 x D block of x (contiguous in HBM) was loaded into registers during the
//              previous iteration; form y = s (x - o) and store it row-major in the wave's LDS
//              slice, then immediately issue the loads of the wave's next row group so that
//              HBM traffic overlaps everything below;
//   2. rotate  Z^T = Qp Y^T on the matrix cores over the nonzero tiles of the packed
//              block-diagonal rotation (Sec. 1.2: three random variable groups, one orthonormal
//              block each).  The B operand is gathered from LDS in group order; on the split
//              paths each y is cut into bf16 terms and the products accumulate in FP32;
//   3. phi     add the offset c and apply the formula straight from the accumulator fragment
//              (pairwise families first exchange z through LDS to reach z_{i+1});
//   4. reduce  per-lane compensated sums, a two-step cross-lane combine, finalise, store.
// The rotation tiles and per-position tables sit in LDS once per workgroup.
#pragma once

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
struct PathT {
  using T = float;
  using V = f32x4;  // 16-byte staging vector
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

// Registers holding one wave's 16 x D slice of x between its load and its staging.
template <int P>
struct XTile {
  using T = typename PathT<P>::T;
  using V = typename PathT<P>::V;
  static constexpr int NV = 16 / sizeof(T);
  static constexpr int TMAX = (kRowsPerWave * 16 * kMaxMT) / (64 * NV);
  V v[TMAX];

  // 16-byte loads of elements (lane + 64 t) * NV < tot of the row group at xg
  __device__ __forceinline__ void load(const T *__restrict__ xg, int tot, int lane) {
#pragma unroll
    for (int t = 0; t < TMAX; ++t) {
      const int e = (lane + 64 * t) * NV;
      if (e < tot) v[t] = __builtin_nontemporal_load(reinterpret_cast<const V *>(xg + e));
    }
  }

  // Y[r][j] = s_j ((x[r][j] - o_j) - olo_j); FP32 paths subtract o as a hi + lo pair so that
  // x - o_hi is exact near the optimum and y keeps its relative accuracy there.
  __device__ __forceinline__ void stage(int tot, int D, int S, T *Y, const T *so, const T *sol, const T *ss,
                                        int lane) const {
    const int e0 = lane * NV;
    int rr = e0 / D, jj = e0 - rr * D;
    constexpr int step = 64 * NV;
    const int dr = step / D, dj = step - dr * D;
#pragma unroll
    for (int t = 0; t < TMAX; ++t) {
      const int e = (lane + 64 * t) * NV;
      if (e < tot) {
        V d = v[t] - *reinterpret_cast<const V *>(so + jj);
        if constexpr (P != PATH_F64) d -= *reinterpret_cast<const V *>(sol + jj);
        *reinterpret_cast<V *>(Y + rr * S + jj) = *reinterpret_cast<const V *>(ss + jj) * d;
      }
      jj += dj;
      rr += dr;
      if (jj >= D) {
        jj -= D;
        ++rr;
      }
    }
  }
};

// Element-wise fallback for dimensions that are not a multiple of the vector width or for
// x pointers that are not 16-byte aligned.
template <int P>
struct XTileScalar {
  using T = typename PathT<P>::T;
  static constexpr int TMAX = (kRowsPerWave * 16 * kMaxMT) / 64;
  T v[TMAX];
  __device__ __forceinline__ void load(const T *__restrict__ xg, int tot, int lane) {
#pragma unroll
    for (int t = 0; t < TMAX; ++t) {
      const int e = lane + 64 * t;
      if (e < tot) v[t] = __builtin_nontemporal_load(xg + e);
    }
  }
  __device__ __forceinline__ void stage(int tot, int D, int S, T *Y, const T *so, const T *sol, const T *ss,
                                        int lane) const {
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
};

// Z^T = Qp Y^T for the wave's 16 rows into acc; element e of acc[m] is packed position
// frag_pos(m, q, e).
template <int P>
__device__ __forceinline__ void rotate(typename PathT<P>::Acc4 (&acc)[kMaxMT], const DevProb &pb,
                                       const unsigned char *s_q, const uint16_t *s_orig,
                                       const typename PathT<P>::T *Yr, int q, int lane) {
  using T = typename PathT<P>::T;
  using Acc4 = typename PathT<P>::Acc4;
#pragma unroll
  for (int m = 0; m < kMaxMT; ++m) acc[m] = Acc4{0, 0, 0, 0};
  const int4 *ktab = reinterpret_cast<const int4 *>(pb.ktab);
  for (int kt = 0; kt < pb.KT; ++kt) {
    const int4 ki = ktab[kt];  // uniform: scalar load
    if constexpr (P == PATH_SPLIT || P == PATH_SPLIT6) {
      // this lane's 8 inputs: packed positions 32 kt + 8 q + 0..7, cut into bf16 terms
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
            // the six products of total order <= 2 in the 2^-8 splitting, smallest first
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
}

template <int P, int KIND, int ROT, typename Tile>
__device__ __forceinline__ void eval_body(const DevProb &pb, const typename PathT<P>::T *__restrict__ x,
                                          typename PathT<P>::T *__restrict__ out, int n) {
  using T = typename PathT<P>::T;
  using Acc4 = typename PathT<P>::Acc4;
  extern __shared__ __align__(16) unsigned char smem[];
  const LdsLayout L = lds_layout(P, pb, blockDim.x >> 6);
  unsigned char *s_q = smem + L.q;
  T *s_o = reinterpret_cast<T *>(smem + L.o);
  T *s_ol = reinterpret_cast<T *>(smem + L.olo);
  T *s_s = reinterpret_cast<T *>(smem + L.s);
  uint16_t *s_orig = reinterpret_cast<uint16_t *>(smem + L.orig);
  T *s_coef = reinterpret_cast<T *>(smem + L.coef);
  T *s_cz = reinterpret_cast<T *>(smem + L.cz);
  int16_t *s_succ = reinterpret_cast<int16_t *>(smem + L.succ);
  T *s_y = reinterpret_cast<T *>(smem + L.y);

  const int D = pb.D, S = pb.S, MT = pb.MT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  const int ngroups = (n + kRowsPerWave - 1) / kRowsPerWave;
  const int gstride = gridDim.x * nwaves;
  int g = blockIdx.x * nwaves + wave;

  // first row group's loads go out before the tables are copied
  Tile xt;
  if (g < ngroups) {
    const int row0 = g * kRowsPerWave;
    xt.load(x + static_cast<size_t>(row0) * D, min(kRowsPerWave, n - row0) * D, lane);
  }
  if (ROT) {
    copy_to_lds(s_q, pb.qfrag, L.q_bytes);
    copy_to_lds(reinterpret_cast<unsigned char *>(s_orig), pb.orig, L.orig_bytes);
  }
  copy_to_lds(reinterpret_cast<unsigned char *>(s_o), pb.o, L.vec_bytes);
  if (P != PATH_F64) copy_to_lds(reinterpret_cast<unsigned char *>(s_ol), pb.olo, L.vec_bytes);
  copy_to_lds(reinterpret_cast<unsigned char *>(s_s), pb.sj, L.vec_bytes);
  if (KindTraits<KIND>::needs_coef) copy_to_lds(reinterpret_cast<unsigned char *>(s_coef), pb.coef, L.mp_bytes);
  copy_to_lds(reinterpret_cast<unsigned char *>(s_cz), pb.cz, L.mp_bytes);
  if (KindTraits<KIND>::pairwise) copy_to_lds(reinterpret_cast<unsigned char *>(s_succ), pb.succ, L.succ_bytes);
  __syncthreads();

  T *Y = s_y + wave * kRowsPerWave * S;
  const T *Yr = Y + r * S;
  if (lane < kRowsPerWave) Y[lane * S + D] = T(0);  // padding slot read by the gather
  const T prm = kind_param<KIND, T>(pb.Df, pb.kparam);

  for (; g < ngroups; g += gstride) {
    const int row0 = g * kRowsPerWave;
    const int nrows = min(kRowsPerWave, n - row0);
    wave_sync();
    xt.stage(nrows * D, D, S, Y, s_o, s_ol, s_s, lane);
    // next row group's loads are in flight during everything below
    const int gn = g + gstride;
    if (gn < ngroups) {
      const int rown = gn * kRowsPerWave;
      xt.load(x + static_cast<size_t>(rown) * D, min(kRowsPerWave, n - rown) * D, lane);
    }
    wave_sync();

    Acc4 acc[kMaxMT];
    if constexpr (ROT) {
      rotate<P>(acc, pb, s_q, s_orig, Yr, q, lane);
    } else {
#pragma unroll
      for (int m = 0; m < kMaxMT; ++m)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int p = frag_pos<P>(m, q, e);
          acc[m][e] = (m < MT && p < D) ? Yr[p] : T(0);
        }
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
          if (m < MT && p < D) Y[r * S + p] = acc[m][e] + s_cz[p];
        }
      wave_sync();
#pragma unroll
      for (int m = 0; m < kMaxMT; ++m)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int p = frag_pos<P>(m, q, e);
          if (m < MT && p < D) {
            const int sp = s_succ[p];
            if (sp >= 0) phi<KIND, T>(a, Yr[p], Yr[sp], T(0), prm);
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
            phi<KIND, T>(a, T(acc[m][e]) + s_cz[p], T(0), cf, prm);
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

template <int P, int KIND, int ROT, int VEC>
__global__ __launch_bounds__(512) void k_eval_resident(DevProb pb, const typename PathT<P>::T *__restrict__ x,
                                                       typename PathT<P>::T *__restrict__ out, int n) {
  if constexpr (VEC)
    eval_body<P, KIND, ROT, XTile<P>>(pb, x, out, n);
  else
    eval_body<P, KIND, ROT, XTileScalar<P>>(pb, x, out, n);
}

// Kernel table of one path: index ((kind * 2) + rot) * 2 + vec.
template <int P, int... Ks>
const void *const *resident_table(std::integer_sequence<int, Ks...>) {
  static const void *const tab[] = {
      (reinterpret_cast<const void *>(&k_eval_resident<P, Ks / 4, (Ks / 2) % 2, Ks % 2>))...};
  return tab;
}

}  // namespace curob
