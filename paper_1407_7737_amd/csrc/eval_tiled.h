// eval_tiled.h -- kernels of the tiled path (see tiled.h for the decomposition).
//
// k_tiled_partial: one workgroup = 64 population rows x one output group (up to four m-tiles of
//   16 outputs, one per wave) of one rotation block.  Per 32-position k step all threads gather
//   y = x - o_hi of the step's variables for the 64 rows into LDS (split paths: already cut into
//   bf16 terms in MFMA B-operand order), then each wave accumulates its m-tile for the four
//   16-row column blocks with A tiles streamed from L2.  The epilogue applies the formula and
//   leaves compensated per-row partial sums of the group in the scratch buffer (pairwise
//   families store z instead).
// k_tiled_finalize: one wave per row combines the partials of each formula segment (and, for
//   pairwise segments, sums the neighbour terms from z), finalises and adds f_opt.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "devprob.h"
#include "formulas.h"
#include "tiled.h"

namespace curob {

namespace tiled {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int P>
struct Types {
  using T = float;
  using Acc4 = f32x4;
};
template <>
struct Types<PATH_F64> {
  using T = double;
  using Acc4 = f64x4;
};

constexpr int kStride = 36;  // LDS row stride (elements) of the FP32/FP64 staging tile

template <int P>
__host__ __device__ constexpr int stage_bytes() {
  return is_split(P) ? split_terms(P) * 4 * 64 * 16 : kTileRows * kStride * (P == PATH_F64 ? 8 : 4);
}
template <int P>
__host__ __device__ constexpr int reduce_bytes() {
  return kGroupMTiles * kTileRows * kPartialSlots * (P == PATH_F64 ? 8 : 4);
}

template <int P>
__device__ __forceinline__ int frag_pos(int q, int e) {
  if constexpr (P == PATH_F64) return 4 * e + q;
  else return 4 * q + e;
}

// The formula of a runtime family id (hybrid segments): one switch per call site.
template <typename T>
__device__ __forceinline__ void phi_any(int kind, T (&v)[3], T &p, T z, T zn, T coef, T prm) {
  switch (kind) {
#define CUROB_PHI_CASE(K) \
  case K: phi<K, T>(v, p, z, zn, coef, prm); break;
    CUROB_PHI_CASE(K_WSPHERE) CUROB_PHI_CASE(K_POWERS) CUROB_PHI_CASE(K_SHARPV) CUROB_PHI_CASE(K_STEP)
    CUROB_PHI_CASE(K_WEIERSTRASS) CUROB_PHI_CASE(K_GRIEWANK) CUROB_PHI_CASE(K_RASTRIGIN) CUROB_PHI_CASE(K_F7)
    CUROB_PHI_CASE(K_GRIEROSEN) CUROB_PHI_CASE(K_ROSENBROCK) CUROB_PHI_CASE(K_SCHWEFEL) CUROB_PHI_CASE(K_KATSUURA)
    CUROB_PHI_CASE(K_LUNACEK) CUROB_PHI_CASE(K_ACKLEY) CUROB_PHI_CASE(K_HAPPYCAT) CUROB_PHI_CASE(K_HGBAT)
    CUROB_PHI_CASE(K_F6)
#undef CUROB_PHI_CASE
    default: break;
  }
}

template <typename T>
__device__ __forceinline__ T finalize_any(int kind, const T (&s)[3], T p, int n) {
  switch (kind) {
#define CUROB_FIN_CASE(K) \
  case K: return finalize<K, T>(s, p, n);
    CUROB_FIN_CASE(K_WSPHERE) CUROB_FIN_CASE(K_POWERS) CUROB_FIN_CASE(K_SHARPV) CUROB_FIN_CASE(K_STEP)
    CUROB_FIN_CASE(K_WEIERSTRASS) CUROB_FIN_CASE(K_GRIEWANK) CUROB_FIN_CASE(K_RASTRIGIN) CUROB_FIN_CASE(K_F7)
    CUROB_FIN_CASE(K_GRIEROSEN) CUROB_FIN_CASE(K_ROSENBROCK) CUROB_FIN_CASE(K_SCHWEFEL) CUROB_FIN_CASE(K_KATSUURA)
    CUROB_FIN_CASE(K_LUNACEK) CUROB_FIN_CASE(K_ACKLEY) CUROB_FIN_CASE(K_HAPPYCAT) CUROB_FIN_CASE(K_HGBAT)
    CUROB_FIN_CASE(K_F6)
#undef CUROB_FIN_CASE
    default: return T(0);
  }
}

template <typename T>
__device__ __forceinline__ T param_any(int kind, int n, double kparam) {
  if (kind == K_SCHWEFEL) return T(1.0 / (10000.0 * (double)n));
  if (kind == K_KATSUURA) return T(kparam);
  return T(0);
}

__device__ __forceinline__ int nsum_any(int kind) {
  return kind == K_LUNACEK ? 3
         : (kind == K_SHARPV || kind == K_ACKLEY || kind == K_HAPPYCAT || kind == K_HGBAT) ? 2
         : kind == K_KATSUURA ? 0
                              : 1;
}

// Formula and row sums of one wave's m-tile for its four 16-row column blocks; the four lanes
// of a row combine their sums and lane group 0 leaves them in the wave's LDS slots.
template <int P, int K>
__device__ __forceinline__ void reduce_tile(const typename Types<P>::Acc4 (&acc)[4], const typename Types<P>::T (&zc)[4],
                                            const typename Types<P>::T (&cf)[4], typename Types<P>::T prm,
                                            typename Types<P>::T *red, int r, int q) {
  using T = typename Types<P>::T;
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    Acc<T> a;
    a.init();
    T v[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int e = 0; e < 4; ++e) phi<K, T>(v, a.p, T(acc[cb][e]) + zc[e], T(0), cf[e], prm);
#pragma unroll
    for (int k = 0; k < 3; ++k) a.add(k, v[k]);
#pragma unroll
    for (int sh = 16; sh <= 32; sh <<= 1) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const T so = __shfl_xor(a.s[k], sh, 64);
        const T co = __shfl_xor(a.c[k], sh, 64);
        acc_merge(a, k, so, co);
      }
      a.p *= __shfl_xor(a.p, sh, 64);
    }
    if (q == 0) {
      T *dst = red + (16 * cb + r) * kPartialSlots;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        dst[2 * k] = a.s[k];
        dst[2 * k + 1] = a.c[k];
      }
      dst[6] = a.p;
    }
  }
}

// KIND >= 0: one formula family for every segment (basic functions); KIND < 0: the family of
// each output group's segment is read at run time (hybrids).
template <int P, int KIND>
__global__ __launch_bounds__(256) void k_tiled_partial(TiledProb tp, const typename Types<P>::T *__restrict__ x, int n,
                                                       typename Types<P>::T *__restrict__ partials,
                                                       typename Types<P>::T *__restrict__ zbuf) {
  using T = typename Types<P>::T;
  using Acc4 = typename Types<P>::Acc4;
  __shared__ __align__(16) unsigned char s_stage[stage_bytes<P>()];
  __shared__ __align__(16) T s_red[kGroupMTiles * kTileRows * kPartialSlots];

  const int4 grp = tp.groups[blockIdx.x];  // block, first m-tile, m-tiles, segment
  const int4 blk = tp.blocks[grp.x];       // padded offset, padded size, first tile, k-tiles
  const TiledSeg &sg = tp.segs[grp.w];
  const int kind = KIND >= 0 ? KIND : sg.kind;
  const int row0 = blockIdx.y * kTileRows;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r = lane & 15, q = lane >> 4;
  const bool active = wave < grp.z;
  const int ml = grp.y + wave;  // this wave's m-tile within the block
  const int D = tp.D;
  const T *oh = reinterpret_cast<const T *>(tp.oh);

  Acc4 acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = Acc4{0, 0, 0, 0};

  // staging assignment: thread -> (row, 8 consecutive positions of the 32-position step)
  const int srow = tid >> 2, sk8 = (tid & 3) * 8;
  const bool srow_ok = row0 + srow < n;
  const T *xrow = x + static_cast<size_t>(row0 + (srow_ok ? srow : 0)) * D;
  const int nsteps = blk.y / kTileK;
  for (int c = 0; c < nsteps; ++c) {
    const int pbase = blk.x + c * kTileK + sk8;
    T y[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int j = tp.gidx[pbase + e];
      y[e] = (j >= 0 && srow_ok) ? xrow[j] - oh[j] : T(0);
    }
    if constexpr (is_split(P)) {
      bf16x8 *st = reinterpret_cast<bf16x8 *>(s_stage);
      const int cb = srow >> 4, slot = (srow & 15) + 16 * (tid & 3);
      bf16x8 h, m, l;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const __bf16 hh = (__bf16)y[e];
        const float r1 = y[e] - (float)hh;
        h[e] = hh;
        if constexpr (P == PATH_SPLIT6) {
          const __bf16 mm = (__bf16)r1;
          m[e] = mm;
          l[e] = (__bf16)(r1 - (float)mm);
        } else {
          l[e] = (__bf16)r1;
        }
      }
      st[(0 * 4 + cb) * 64 + slot] = h;
      if constexpr (P == PATH_SPLIT6) {
        st[(1 * 4 + cb) * 64 + slot] = m;
        st[(2 * 4 + cb) * 64 + slot] = l;
      } else {
        st[(1 * 4 + cb) * 64 + slot] = l;
      }
    } else {
      T *st = reinterpret_cast<T *>(s_stage) + srow * kStride + sk8;
#pragma unroll
      for (int e = 0; e < 8; ++e) st[e] = y[e];
    }
    __syncthreads();
    if (active) {
      if constexpr (is_split(P)) {
        constexpr int NT = split_terms(P);
        const int t = blk.z + ml * blk.w + c;  // split k-tiles are the 32-position steps
        const bf16x8 *qf = reinterpret_cast<const bf16x8 *>(tp.qfrag) + static_cast<size_t>(t) * NT * 64 + lane;
        const bf16x8 *st = reinterpret_cast<const bf16x8 *>(s_stage);
        const bf16x8 ah = qf[0];
        const bf16x8 a2 = qf[64];
        bf16x8 a3;
        if constexpr (NT == 3) a3 = qf[128];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          const bf16x8 bh = st[(0 * 4 + cb) * 64 + lane];
          const bf16x8 b2 = st[(1 * 4 + cb) * 64 + lane];
          if constexpr (NT == 3) {
            // terms hi, mid, lo: the six products of order <= 2
            const bf16x8 b3 = st[(2 * 4 + cb) * 64 + lane];
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3, bh, acc[cb], 0, 0, 0);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b2, acc[cb], 0, 0, 0);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b3, acc[cb], 0, 0, 0);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, bh, acc[cb], 0, 0, 0);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b2, acc[cb], 0, 0, 0);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[cb], 0, 0, 0);
          } else {
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, bh, acc[cb], 0, 0, 0);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b2, acc[cb], 0, 0, 0);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[cb], 0, 0, 0);
          }
        }
      } else {
        const T *st = reinterpret_cast<const T *>(s_stage);
        const T *qf = reinterpret_cast<const T *>(tp.qfrag);
#pragma unroll
        for (int s4 = 0; s4 < kTileK / 4; ++s4) {
          const int t = blk.z + ml * blk.w + c * (kTileK / 4) + s4;
          const T a = qf[static_cast<size_t>(t) * 64 + lane];
#pragma unroll
          for (int cb = 0; cb < 4; ++cb) {
            const T b = st[(16 * cb + r) * kStride + 4 * s4 + q];
            if constexpr (P == PATH_F64)
              acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[cb], 0, 0, 0);
            else
              acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[cb], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }

  // epilogue
  const T *cz = reinterpret_cast<const T *>(tp.cz);
  const T *coefp = reinterpret_cast<const T *>(tp.coef);
  const int pm = blk.x + 16 * ml;  // first padded position of this wave's m-tile
  T *red = s_red + (wave * kTileRows) * kPartialSlots;
  if (active) {
    if (sg.pairwise) {
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const int row = row0 + 16 * cb + r;
        if (row < n) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int pp = pm + frag_pos<P>(q, e);
            zbuf[static_cast<size_t>(row) * tp.Dp + pp] = T(acc[cb][e]) + cz[pp];
          }
        }
      }
    } else {
      T zc[4], cf[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int pp = pm + frag_pos<P>(q, e);
        zc[e] = cz[pp];
        cf[e] = coefp[pp];
      }
      if constexpr (KIND >= 0) {
        reduce_tile<P, KIND>(acc, zc, cf, kind_param<KIND, T>(sg.n, sg.kparam), red, r, q);
      } else {
        // hybrids: one branch per wave on the segment's family
        const T prm = param_any<T>(kind, sg.n, sg.kparam);
        switch (kind) {
#define CUROB_RT_CASE(K) \
  case K: reduce_tile<P, K>(acc, zc, cf, prm, red, r, q); break;
          CUROB_RT_CASE(K_WSPHERE) CUROB_RT_CASE(K_POWERS) CUROB_RT_CASE(K_SHARPV) CUROB_RT_CASE(K_STEP)
          CUROB_RT_CASE(K_WEIERSTRASS) CUROB_RT_CASE(K_GRIEWANK) CUROB_RT_CASE(K_RASTRIGIN)
          CUROB_RT_CASE(K_SCHWEFEL) CUROB_RT_CASE(K_KATSUURA) CUROB_RT_CASE(K_LUNACEK) CUROB_RT_CASE(K_ACKLEY)
          CUROB_RT_CASE(K_HAPPYCAT) CUROB_RT_CASE(K_HGBAT)
#undef CUROB_RT_CASE
          default: break;  // pairwise families store z above
        }
      }
    }
  }
  __syncthreads();
  if (!sg.pairwise && tid < kTileRows && row0 + tid < n) {
    // combine the output group's m-tiles for row tid
    Acc<T> a;
    a.init();
    for (int w = 0; w < grp.z; ++w) {
      const T *src = s_red + (w * kTileRows + tid) * kPartialSlots;
#pragma unroll
      for (int k = 0; k < 3; ++k) acc_merge(a, k, src[2 * k], src[2 * k + 1]);
      a.p *= src[6];
    }
    T *dst = partials + (static_cast<size_t>(blockIdx.x) * kChunkRows + row0 + tid) * kPartialSlots;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      dst[2 * k] = a.s[k];
      dst[2 * k + 1] = a.c[k];
    }
    dst[6] = a.p;
  }
}

// One wave per row: combine the segments' partials, add pairwise terms, finalise.
template <int P>
__global__ __launch_bounds__(256) void k_tiled_finalize(TiledProb tp, const typename Types<P>::T *__restrict__ partials,
                                                        const typename Types<P>::T *__restrict__ zbuf, int n,
                                                        typename Types<P>::T *__restrict__ out) {
  using T = typename Types<P>::T;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (row >= n) return;
  T F = T(0);
  const T *coefp = reinterpret_cast<const T *>(tp.coef);
  for (int si = 0; si < tp.nsegs; ++si) {
    const TiledSeg &sg = tp.segs[si];
    Acc<T> a;
    a.init();
    if (sg.pairwise) {
      const T prm = param_any<T>(sg.kind, sg.n, sg.kparam);
      const T *zr = zbuf + static_cast<size_t>(row) * tp.Dp;
      for (int pp = sg.p0 + lane; pp < sg.p1; pp += 64) {
        const int sp = tp.succ[pp];
        if (tp.gidx[pp] >= 0 && sp >= 0) {
          T v[3] = {T(0), T(0), T(0)};
          phi_any<T>(sg.kind, v, a.p, zr[pp], zr[sp], coefp[pp], prm);
          a.add(0, v[0]);
        }
      }
#pragma unroll
      for (int sh = 1; sh < 64; sh <<= 1) {
        const T so = __shfl_xor(a.s[0], sh, 64);
        const T co = __shfl_xor(a.c[0], sh, 64);
        acc_merge(a, 0, so, co);
      }
    } else if (lane == 0) {
      for (int g = sg.g0; g < sg.g1; ++g) {
        const T *src = partials + (static_cast<size_t>(g) * kChunkRows + row) * kPartialSlots;
#pragma unroll
        for (int k = 0; k < 3; ++k) acc_merge(a, k, src[2 * k], src[2 * k + 1]);
        a.p *= src[6];
      }
    }
    if (lane == 0) {
      T s[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) s[k] = a.get(k) - T(sg.padc[k]);
      F += finalize_any<T>(sg.kind, s, a.p, sg.n);
    }
  }
  if (lane == 0) out[row] = F + T(tp.bias);
}

}  // namespace tiled

}  // namespace curob
