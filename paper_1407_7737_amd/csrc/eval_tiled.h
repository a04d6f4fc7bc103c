// eval_tiled.h -- kernels of the tiled path (see tiled.h for the decomposition).
//
// k_tiled_pack: one workgroup stages R consecutive population rows (coalesced) in LDS and
//   writes y = x - o_hi of every 32-position k step in packed (group) order, already in MFMA
//   B-operand layout and, on the split paths, cut into bf16 terms: per (16-row tile, k step) a
//   chunk of parts x 64 lanes x 16 bytes that a wave reads with one 16-byte load per part.
// k_tiled_gemm: one workgroup = 64 rows (four row tiles) x one output group (up to four
//   m-tiles of 16 outputs, one per wave) of one rotation block.  The chunks of the next k
//   step are loaded into registers while the current step's MFMAs run on the other LDS buffer
//   (one barrier per step); rotation tiles come from L2.  The epilogue applies the formula and
//   leaves compensated per-row partial sums of the group in scratch (pairwise families store
//   z instead).
// k_tiled_finalize: one thread per row combines the partials of each formula segment,
//   finalises and adds f_opt; k_tiled_finalize_pairs does the same with one wave per row for
//   problems with pairwise segments, whose neighbour terms are summed from z.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

#include "devprob.h"
#include "formulas.h"
#include "kernels.h"
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

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// 16-byte parts per lane of a pack chunk: the bf16 terms on the split paths (8 positions
// each), the eight 4-position k tiles of a step as 2 x 4 floats or 4 x 2 doubles.
template <int P>
__host__ __device__ constexpr int pack_parts() {
  return is_split(P) ? split_terms(P) : (P == PATH_F64 ? 4 : 2);
}
template <int P>
__host__ __device__ constexpr int chunk_bytes() {
  return pack_parts<P>() * 64 * 16;
}

// Each of the four waves computes kWaveM m-tiles x kWaveR row tiles of the workgroup's
// kGroupMTiles x kRowTiles: every B fragment read from LDS feeds kWaveM m-tiles.
constexpr int kWaveM = 2;
constexpr int kWaveR = 4;
constexpr int kGemmWaves = kGroupMTiles / kWaveM * (kRowTiles / kWaveR);
constexpr int kGemmThreads = 64 * kGemmWaves;

template <int P>
__device__ __forceinline__ int frag_pos(int q, int e) {
  if constexpr (P == PATH_F64) return 4 * e + q;
  else return 4 * q + e;
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

// Formula and row sums of one m-tile of a wave for its four 16-row column blocks; the four
// lanes of a row combine their sums and lane group 0 leaves them in the m-tile's LDS slots.
template <int P, int K>
__device__ __forceinline__ void reduce_tile(const typename Types<P>::Acc4 (&acc)[kWaveR], const typename Types<P>::T (&zc)[4],
                                            const typename Types<P>::T (&cf)[4], typename Types<P>::T prm,
                                            typename Types<P>::T *red, int r, int q) {
  using T = typename Types<P>::T;
#pragma unroll
  for (int cb = 0; cb < kWaveR; ++cb) {
    Acc<T> a;
    a.init();
    T v[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int e = 0; e < 4; ++e) phi<K, T>(v, a.p, T(acc[cb][e]) + zc[e], T(0), cf[e], prm);
#pragma unroll
    for (int k = 0; k < 3; ++k) acc_add<K, T>(a, k, v[k]);
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

// Pack chunk of row tile rt, global k step c: chunk index rt * nsteps + c.
template <int P>
__global__ __launch_bounds__(256) void k_tiled_pack(TiledProb tp, const typename Types<P>::T *__restrict__ x, int n,
                                                    int rows_per_wg, int SX, int vec, unsigned char *__restrict__ pack) {
  using T = typename Types<P>::T;
  constexpr int NP = pack_parts<P>();
  extern __shared__ __align__(16) unsigned char smem[];
  const int D = tp.D, R = rows_per_wg;
  const int nsteps = tp.Dp / kTileK;
  int *s_gidx = reinterpret_cast<int *>(smem);
  T *s_oh = reinterpret_cast<T *>(smem + round16(tp.Dp * 4));
  T *s_x = reinterpret_cast<T *>(smem + round16(tp.Dp * 4) + round16(D * static_cast<int>(sizeof(T))));
  const int row0 = blockIdx.x * R;  // rows [row0, row0 + R) lie in one row tile
  const int nvalid = n - row0 < 0 ? 0 : (n - row0 < R ? n - row0 : R);
  // position tables: a thread's loads of a round are issued before its stores (clamped
  // indices, no branch around a load), so the copy costs one memory round trip per round
  for (int base = threadIdx.x; base < tp.Dp; base += 256 * 4) {
    int g[4];
    T oh4[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = base + 256 * u;
      g[u] = tp.gidx[i < tp.Dp ? i : tp.Dp - 1];
      oh4[u] = reinterpret_cast<const T *>(tp.oh)[i < D ? i : D - 1];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = base + 256 * u;
      if (i < tp.Dp) s_gidx[i] = g[u];
      if (i < D) s_oh[i] = oh4[u];
    }
  }
  // stage the rows at stride SX (the 16 rows of a tile fall in distinct LDS banks); all of a
  // thread's loads are issued before any store so many requests are in flight
  constexpr int U = 16;
  const T *xs = x + static_cast<size_t>(row0) * D;
  if (vec) {
    // rows of 16-byte multiples, 16-byte aligned: vector loads
    constexpr int NV = 16 / static_cast<int>(sizeof(T));
    using V = typename std::conditional<sizeof(T) == 8, f64x2, f32x4>::type;
    const V *xv = reinterpret_cast<const V *>(xs);
    const int DV = D / NV, tv = R * DV, vv = nvalid * DV;
    for (int base = 0; base < tv; base += 256 * U) {
      V v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = base + 256 * u + threadIdx.x;
        v[u] = i < vv ? xv[i] : V{};
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = base + 256 * u + threadIdx.x;
        if (i < tv) {
          const int row = i / DV;
          *reinterpret_cast<V *>(s_x + row * SX + (i - row * DV) * NV) = v[u];
        }
      }
    }
  } else {
    const int total = R * D, valid = nvalid * D;
    for (int base = 0; base < total; base += 256 * U) {
      T v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = base + 256 * u + threadIdx.x;
        v[u] = i < valid ? xs[i] : T(0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = base + 256 * u + threadIdx.x;
        if (i < total) {
          const int row = i / D;
          s_x[row * SX + (i - row * D)] = v[u];
        }
      }
    }
  }
  __syncthreads();

  const int rt = row0 / 16, r0 = row0 % 16;
  const int items = nsteps * 4 * R;
  for (int it = threadIdx.x; it < items; it += 256) {
    const int c = it / (4 * R), rem = it - c * (4 * R);
    const int g = rem / R, r = r0 + rem % R;
    const int lane = r + 16 * g;
    const T *xr = s_x + (r - r0) * SX;
    const bool live = r - r0 < nvalid;
    unsigned char *dst = pack + (static_cast<size_t>(rt) * nsteps + c) * chunk_bytes<P>() + lane * 16;
    T y[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      // split: positions 8g + e of the step; FP32/FP64: position 4e + g (k tile e, row g of it)
      const int pos = c * kTileK + (is_split(P) ? 8 * g + e : 4 * e + g);
      const int j = s_gidx[pos];
      y[e] = (j >= 0 && live) ? xr[j] - s_oh[j] : T(0);
    }
    if constexpr (is_split(P)) {
      bf16x8 t0, t1, t2;
#pragma unroll
      for (int e = 0; e < 8; e += 2) {
        const f32x2 v = {y[e], y[e + 1]};
        const bf16x2 h = __builtin_convertvector(v, bf16x2);
        const f32x2 r1 = v - __builtin_convertvector(h, f32x2);
        t0[e] = h[0];
        t0[e + 1] = h[1];
        if constexpr (NP == 3) {
          const bf16x2 m = __builtin_convertvector(r1, bf16x2);
          const bf16x2 l = __builtin_convertvector(r1 - __builtin_convertvector(m, f32x2), bf16x2);
          t1[e] = m[0];
          t1[e + 1] = m[1];
          t2[e] = l[0];
          t2[e + 1] = l[1];
        } else {
          const bf16x2 l = __builtin_convertvector(r1, bf16x2);
          t1[e] = l[0];
          t1[e + 1] = l[1];
        }
      }
      *reinterpret_cast<bf16x8 *>(dst) = t0;
      *reinterpret_cast<bf16x8 *>(dst + 1024) = t1;
      if constexpr (NP == 3) *reinterpret_cast<bf16x8 *>(dst + 2048) = t2;
    } else if constexpr (P == PATH_F64) {
#pragma unroll
      for (int pt = 0; pt < 4; ++pt) *reinterpret_cast<f64x2 *>(dst + pt * 1024) = f64x2{y[2 * pt], y[2 * pt + 1]};
    } else {
      *reinterpret_cast<f32x4 *>(dst) = f32x4{y[0], y[1], y[2], y[3]};
      *reinterpret_cast<f32x4 *>(dst + 1024) = f32x4{y[4], y[5], y[6], y[7]};
    }
  }
}

template <int P>
using AFragT = typename std::conditional<is_split(P), bf16x8, typename Types<P>::T>::type;
template <int P>
constexpr int kNA = is_split(P) ? split_terms(P) : 8;  // A fragments per step
template <int P>
constexpr int kPT = kRowTiles * pack_parts<P>() * 64 / kGemmThreads;  // 16-byte B pieces per thread per step

// One k step of the GEMM: issue the loads of step c + 2 into (rl, au after use), run step c's
// MFMAs from LDS buffer c & 1 with the rotation tiles au, store step c + 1 (rw) into the other
// buffer, barrier.
template <int P>
__device__ __forceinline__ void gemm_step(int c, int nst, const unsigned char *src0, const size_t (&src_off)[kPT<P>],
                                          unsigned char *s_mem, int tid, int lane, int rq,
                                          const AFragT<P> *const (&qa)[kWaveM], u32x4 (&rl)[kPT<P>],
                                          const u32x4 (&rw)[kPT<P>], AFragT<P> (&au)[kWaveM][kNA<P>],
                                          typename Types<P>::Acc4 (&acc)[kWaveM][kWaveR]) {
  using T = typename Types<P>::T;
  constexpr int CH = chunk_bytes<P>();
  constexpr int BUF = kRowTiles * CH;
  constexpr int PT = kPT<P>, NA = kNA<P>;
  // No branches inside a step: the waits on outstanding loads stay exact (a branch makes the
  // compiler wait for every load, the prefetches included).  Past the last step the loads
  // repeat the last step and the stores fill a buffer nobody reads; inactive m-tiles (an
  // odd last group of a block) multiply a valid tile and are discarded.
  const int buf = c & 1;
  const int cn = c + 2 < nst ? c + 2 : nst - 1;
#pragma unroll
  for (int k2 = 0; k2 < PT; ++k2)
    rl[k2] = *reinterpret_cast<const u32x4 *>(src0 + src_off[k2] + static_cast<size_t>(cn) * CH);
  // keep the prefetch loads at the top of the step (the scheduler would otherwise sink them
  // next to the stores that consume them)
  __builtin_amdgcn_sched_barrier(0);
  {
    const unsigned char *sb = s_mem + buf * BUF + kWaveR * rq * CH;
#pragma unroll
    for (int cb = 0; cb < kWaveR; ++cb) {
      if constexpr (is_split(P)) {
        const bf16x8 *bb = reinterpret_cast<const bf16x8 *>(sb + cb * CH) + lane;
        const bf16x8 bh = bb[0];
        const bf16x8 b2 = bb[64];
        bf16x8 b3;
        if constexpr (split_terms(P) == 3) b3 = bb[128];
#pragma unroll
        for (int j = 0; j < kWaveM; ++j) {
          auto &ac = acc[j][cb];
          if constexpr (split_terms(P) == 3) {
            // terms hi, mid, lo: the six products of order <= 2
            ac = __builtin_amdgcn_mfma_f32_16x16x32_bf16(au[j][2], bh, ac, 0, 0, 0);
            ac = __builtin_amdgcn_mfma_f32_16x16x32_bf16(au[j][1], b2, ac, 0, 0, 0);
            ac = __builtin_amdgcn_mfma_f32_16x16x32_bf16(au[j][0], b3, ac, 0, 0, 0);
            ac = __builtin_amdgcn_mfma_f32_16x16x32_bf16(au[j][1], bh, ac, 0, 0, 0);
            ac = __builtin_amdgcn_mfma_f32_16x16x32_bf16(au[j][0], b2, ac, 0, 0, 0);
            ac = __builtin_amdgcn_mfma_f32_16x16x32_bf16(au[j][0], bh, ac, 0, 0, 0);
          } else {
            ac = __builtin_amdgcn_mfma_f32_16x16x32_bf16(au[j][1], bh, ac, 0, 0, 0);
            ac = __builtin_amdgcn_mfma_f32_16x16x32_bf16(au[j][0], b2, ac, 0, 0, 0);
            ac = __builtin_amdgcn_mfma_f32_16x16x32_bf16(au[j][0], bh, ac, 0, 0, 0);
          }
        }
      } else {
        T b[8];
        if constexpr (P == PATH_F64) {
#pragma unroll
          for (int pt = 0; pt < 4; ++pt) {
            const f64x2 v = *reinterpret_cast<const f64x2 *>(sb + cb * CH + pt * 1024 + lane * 16);
            b[2 * pt] = v[0];
            b[2 * pt + 1] = v[1];
          }
        } else {
#pragma unroll
          for (int pt = 0; pt < 2; ++pt) {
            const f32x4 v = *reinterpret_cast<const f32x4 *>(sb + cb * CH + pt * 1024 + lane * 16);
#pragma unroll
            for (int e = 0; e < 4; ++e) b[4 * pt + e] = v[e];
          }
        }
#pragma unroll
        for (int j = 0; j < kWaveM; ++j) {
#pragma unroll
          for (int s4 = 0; s4 < 8; ++s4) {
            if constexpr (P == PATH_F64)
              acc[j][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(au[j][s4], b[s4], acc[j][cb], 0, 0, 0);
            else
              acc[j][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(au[j][s4], b[s4], acc[j][cb], 0, 0, 0);
          }
        }
      }
    }
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int j = 0; j < kWaveM; ++j)
#pragma unroll
    for (int u = 0; u < NA; ++u) au[j][u] = qa[j][(static_cast<size_t>(cn) * NA + u) * 64];
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int k2 = 0; k2 < PT; ++k2)
    *reinterpret_cast<u32x4 *>(s_mem + (buf ^ 1) * BUF + (tid + kGemmThreads * k2) * 16) = rw[k2];
  __syncthreads();
}

// Epilogue of one m-tile (mi within the group) of a wave over its kWaveR row tiles: pairwise
// families store z, the others apply the formula and leave row partials in LDS.
template <int P, int KIND>
__device__ __forceinline__ void mtile_epilogue(const TiledProb &tp, const TiledSeg &sg, int kind, int4 grp, int4 blk,
                                               int mi, int rq, int row0, int n, int r, int q,
                                               const typename Types<P>::Acc4 (&acc)[kWaveR],
                                               typename Types<P>::T *s_red, typename Types<P>::T *zbuf) {
  using T = typename Types<P>::T;
  if (mi >= grp.z) return;
  const T *cz = reinterpret_cast<const T *>(tp.cz);
  const T *coefp = reinterpret_cast<const T *>(tp.coef);
  const int pm = blk.x + 16 * (grp.y + mi);  // first padded position of the m-tile
  if (sg.pairwise) {
#pragma unroll
    for (int cb = 0; cb < kWaveR; ++cb) {
      const int row = row0 + 16 * (kWaveR * rq + cb) + r;
      if (row < n) {
        if constexpr (P == PATH_F64) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int pp = pm + frag_pos<P>(q, e);
            zbuf[static_cast<size_t>(row) * tp.Dp + pp] = T(acc[cb][e]) + cz[pp];
          }
        } else {
          // positions pm + 4 q .. + 3 are consecutive and 16-byte aligned: one vector store
          const int pp = pm + 4 * q;
          const f32x4 c4 = *reinterpret_cast<const f32x4 *>(cz + pp);
          *reinterpret_cast<f32x4 *>(zbuf + static_cast<size_t>(row) * tp.Dp + pp) =
              f32x4{float(acc[cb][0]), float(acc[cb][1]), float(acc[cb][2]), float(acc[cb][3])} + c4;
        }
      }
    }
    return;
  }
  T zc[4], cf[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int pp = pm + frag_pos<P>(q, e);
    zc[e] = cz[pp];
    cf[e] = coefp[pp];
  }
  T *red = s_red + (mi * kTileRows + 16 * kWaveR * rq) * kPartialSlots;
  if constexpr (KIND >= 0) {
    reduce_tile<P, KIND>(acc, zc, cf, kind_param<KIND, T>(sg.n, sg.kparam), red, r, q);
  } else {
    // hybrids: one branch per wave on the segment's family
    const T prm = param_any<T>(kind, sg.n, sg.kparam);
    switch (kind) {
#define CUROB_RT_CASE(K) \
  case K: reduce_tile<P, K>(acc, zc, cf, prm, red, r, q); break;
      CUROB_RT_CASE(K_WSPHERE) CUROB_RT_CASE(K_POWERS) CUROB_RT_CASE(K_SHARPV) CUROB_RT_CASE(K_STEP)
      CUROB_RT_CASE(K_WEIERSTRASS) CUROB_RT_CASE(K_GRIEWANK) CUROB_RT_CASE(K_RASTRIGIN) CUROB_RT_CASE(K_SCHWEFEL)
      CUROB_RT_CASE(K_KATSUURA) CUROB_RT_CASE(K_LUNACEK) CUROB_RT_CASE(K_ACKLEY) CUROB_RT_CASE(K_HAPPYCAT)
      CUROB_RT_CASE(K_HGBAT)
#undef CUROB_RT_CASE
      default: break;  // pairwise families store z above
    }
  }
}

// KIND >= 0: one formula family for every segment (basic functions); KIND < 0: the family of
// each output group's segment is read at run time (hybrids).
template <int P, int KIND>
__global__ __launch_bounds__(kGemmThreads) void k_tiled_gemm(TiledProb tp, const unsigned char *pack, int n,
                                                    int ntiles, typename Types<P>::T *__restrict__ partials,
                                                    typename Types<P>::T *__restrict__ zbuf, int pstride) {
  using T = typename Types<P>::T;
  using Acc4 = typename Types<P>::Acc4;
  constexpr int NP = pack_parts<P>();
  constexpr int CH = chunk_bytes<P>();
  // two step buffers of the workgroup's row tiles; after the k loop the same LDS holds the
  // per-wave partial sums of the epilogue
  constexpr int BUF = kRowTiles * CH;
  constexpr int RED = kGroupMTiles * kTileRows * kPartialSlots * static_cast<int>(sizeof(T));
  __shared__ __align__(16) unsigned char s_mem[2 * BUF > RED ? 2 * BUF : RED];
  T *s_red = reinterpret_cast<T *>(s_mem);

  // Workgroups are dealt to the XCDs round robin; every output group of a row tile is mapped
  // to the same XCD so the tile's packed operands are fetched into one L2 only.
  const int xcd = blockIdx.x % kNumXcd, k = blockIdx.x / kNumXcd;
  const int gi = k % tp.ngroups;
  const int tile = (k / tp.ngroups) * kNumXcd + xcd;
  if (tile >= ntiles) return;  // padding of the grid to whole rounds of XCDs
  const int4 grp = tp.groups[gi];     // block, first m-tile, m-tiles, segment
  const int4 blk = tp.blocks[grp.x];  // padded offset, padded size, first tile, k-tiles
  const TiledSeg &sg = tp.segs[grp.w];
  const int kind = KIND >= 0 ? KIND : sg.kind;
  const int row0 = tile * kTileRows;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r = lane & 15, q = lane >> 4;
  // this wave: m-tiles mi0, mi0 + 1 of the group, row tiles kWaveR rq .. kWaveR rq + 3
  const int mi0 = kWaveM * (wave % (kGroupMTiles / kWaveM)), rq = wave / (kGroupMTiles / kWaveM);
  const int nsteps_all = tp.Dp / kTileK;
  const int c0 = blk.x / kTileK, nst = blk.y / kTileK;

  // one step of the workgroup's row tiles: kRowTiles * NP * 64 pieces of 16 bytes, PT per
  // thread; piece p of the step sits at byte 16 p of the LDS buffer (row tile i at i * CH)
  constexpr int PT = kPT<P>;
  const unsigned char *src0 = pack + (static_cast<size_t>(tile) * kRowTiles * nsteps_all + c0) * CH;
  size_t src_off[PT];
#pragma unroll
  for (int k2 = 0; k2 < PT; ++k2) {
    const int piece = tid + kGemmThreads * k2;
    const int i = piece / (NP * 64), off = piece - i * (NP * 64);
    src_off[k2] = static_cast<size_t>(i) * nsteps_all * CH + off * 16;
  }
  // rotation tiles of this wave's m-tiles (inactive ones read a valid tile and ignore it)
  constexpr int NA = kNA<P>;
  using AFrag = AFragT<P>;
  const AFrag *qa[kWaveM];
#pragma unroll
  for (int j = 0; j < kWaveM; ++j) {
    const int mt = grp.y + (mi0 + j < grp.z ? mi0 + j : 0);
    qa[j] = reinterpret_cast<const AFrag *>(tp.qfrag) +
            static_cast<size_t>(blk.z + mt * blk.w) * (is_split(P) ? split_terms(P) : 1) * 64 + lane;
  }

  // Operands run two steps ahead.  Even steps load into (rb0, a0), odd steps into (rb1, a1):
  // step c's B is in LDS buffer c & 1, step c + 1's in registers, step c + 2's in flight.
  u32x4 rb0[PT], rb1[PT];
  AFrag a0[kWaveM][NA], a1[kWaveM][NA];
#pragma unroll
  for (int k2 = 0; k2 < PT; ++k2) rb0[k2] = *reinterpret_cast<const u32x4 *>(src0 + src_off[k2]);
#pragma unroll
  for (int j = 0; j < kWaveM; ++j)
#pragma unroll
    for (int u = 0; u < NA; ++u) a0[j][u] = qa[j][u * 64];
  if (nst > 1) {
#pragma unroll
    for (int k2 = 0; k2 < PT; ++k2) rb1[k2] = *reinterpret_cast<const u32x4 *>(src0 + src_off[k2] + CH);
#pragma unroll
    for (int j = 0; j < kWaveM; ++j)
#pragma unroll
      for (int u = 0; u < NA; ++u) a1[j][u] = qa[j][(NA + u) * 64];
  }
#pragma unroll
  for (int k2 = 0; k2 < PT; ++k2) *reinterpret_cast<u32x4 *>(s_mem + (tid + kGemmThreads * k2) * 16) = rb0[k2];
  __syncthreads();

  Acc4 acc[kWaveM][kWaveR];
#pragma unroll
  for (int j = 0; j < kWaveM; ++j)
#pragma unroll
    for (int cb = 0; cb < kWaveR; ++cb) acc[j][cb] = Acc4{0, 0, 0, 0};

  for (int c = 0; c < nst; c += 2) {
    gemm_step<P>(c, nst, src0, src_off, s_mem, tid, lane, rq, qa, rb0, rb1, a0, acc);
    if (c + 1 < nst) gemm_step<P>(c + 1, nst, src0, src_off, s_mem, tid, lane, rq, qa, rb1, rb0, a1, acc);
  }

  // epilogue: each of the wave's m-tiles, its four row tiles
  mtile_epilogue<P, KIND>(tp, sg, kind, grp, blk, mi0, rq, row0, n, r, q, acc[0], s_red, zbuf);
  mtile_epilogue<P, KIND>(tp, sg, kind, grp, blk, mi0 + 1, rq, row0, n, r, q, acc[1], s_red, zbuf);
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
    T *dst = partials + (static_cast<size_t>(gi) * pstride + row0 + tid) * kPartialSlots;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      dst[2 * k] = a.s[k];
      dst[2 * k + 1] = a.c[k];
    }
    dst[6] = a.p;
  }
}

// Unrotated basic problems of any dimension: one wave per row streams the row (coalesced),
// forms z = s (x - o_hi) + c' per variable and the formula's terms (the successor's z for the
// pairwise families), sums them compensated per lane, combines the lanes and finalises.
template <int P, int KIND>
__global__ __launch_bounds__(256) void k_rowwise(TiledProb tp, const typename Types<P>::T *__restrict__ x, int n,
                                                 typename Types<P>::T *__restrict__ out) {
  using T = typename Types<P>::T;
  using KT_ = KindTraits<KIND>;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (row >= n) return;
  const int D = tp.D;
  const T s = T(tp.scale0);
  const T *oh = reinterpret_cast<const T *>(tp.oh);
  const T *cz = reinterpret_cast<const T *>(tp.cz);
  const T *coef = reinterpret_cast<const T *>(tp.coef);
  const TiledSeg &sg = tp.segs[0];
  const T prm = kind_param<KIND, T>(sg.n, sg.kparam);
  const T *xr = x + static_cast<size_t>(row) * D;
  Acc<T> a;
  a.init();
  for (int j0 = 0; j0 < D; j0 += 256) {
    // every load of the step is issued before the first use (indices past the row are clamped
    // and their terms masked), so the step waits for memory once
    T xv[4], ov[4], cv[4], fv[4], xn[4], on[4], cn[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + 64 * u + lane;
      const int jc = j < D ? j : D - 1;
      xv[u] = xr[jc];
      ov[u] = oh[jc];
      cv[u] = cz[jc];
      fv[u] = KT_::needs_coef || KT_::pairwise ? coef[jc] : T(0);
      if constexpr (KT_::pairwise) {
        const int jn = jc + 1 < D ? jc + 1 : 0;
        xn[u] = xr[jn];
        on[u] = oh[jn];
        cn[u] = cz[jn];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    T v[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + 64 * u + lane;
      if (j < D) {
        const T z = s * (xv[u] - ov[u]) + cv[u];
        if constexpr (KT_::pairwise) {
          // the last variable pairs with the first only for the wrapping families
          if (j + 1 < D || kind_pair_wraps_c(KIND)) {
            const T zn = s * (xn[u] - on[u]) + cn[u];
            T w[3] = {T(0), T(0), T(0)};
            phi<KIND, T>(w, a.p, z, zn, fv[u], prm);
            v[0] += w[0];
          }
        } else {
          phi<KIND, T>(v, a.p, z, T(0), fv[u], prm);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) acc_add<KIND, T>(a, k, v[k]);
  }
#pragma unroll
  for (int sh = 1; sh < 64; sh <<= 1) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const T so = __shfl_xor(a.s[k], sh, 64);
      const T co = __shfl_xor(a.c[k], sh, 64);
      acc_merge(a, k, so, co);
    }
    if constexpr (KT_::has_product) a.p *= __shfl_xor(a.p, sh, 64);
  }
  if (lane == 0) {
    T sums[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) sums[k] = a.get(k);
    out[row] = finalize<KIND, T>(sums, a.p, D) + T(tp.bias);
  }
}

// One wave per row: combine the segments' partials, add pairwise terms, finalise.
template <int P>
__global__ __launch_bounds__(256) void k_tiled_finalize(TiledProb tp, const typename Types<P>::T *__restrict__ partials,
                                                        const typename Types<P>::T *__restrict__ zbuf, int n,
                                                        typename Types<P>::T *__restrict__ out, int pstride) {
  using T = typename Types<P>::T;
  (void)zbuf;
  // one thread per row (problems without pair terms): the partial slots of consecutive rows
  // are adjacent, so each output group's slots are read as one contiguous run per wave
  const int row = blockIdx.x * 256 + threadIdx.x;
  const bool live = row < n;
  T F = T(0);
  for (int si = 0; si < tp.nsegs; ++si) {
    const TiledSeg &sg = tp.segs[si];
    Acc<T> a;
    a.init();
    if (live) {
      for (int g = sg.g0; g < sg.g1; ++g) {
        const T *src = partials + (static_cast<size_t>(g) * pstride + row) * kPartialSlots;
        T v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = src[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) acc_merge(a, k, v[2 * k], v[2 * k + 1]);
        a.p *= v[6];
      }
    }
    T sm[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) sm[k] = a.get_minus(k, sg.padc[k]);
    F += finalize_any<T>(sg.kind, sm, a.p, sg.n);
  }
  if (live) out[row] = F + T(tp.bias);
}

// Pair terms of one pairwise segment for one row (z in zr, padded order), lanes over the
// positions, two per lane per step: the table and z loads of a step are issued together
// (positions past the segment are clamped and masked), then the formula of family K.
template <int K, typename T>
__device__ __forceinline__ void pair_terms(const TiledProb &tp, const TiledSeg &sg, const T *zr, const T *coefp, T prm,
                                           int lane, Acc<T> &a) {
  for (int p0 = sg.p0; p0 < sg.p1; p0 += 128) {
    int pc[2], sp[2], gi[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int pp = p0 + 64 * u + lane;
      pc[u] = pp < sg.p1 ? pp : sg.p1 - 1;
      sp[u] = tp.succ[pc[u]];
      gi[u] = tp.gidx[pc[u]];
    }
    T z[2], zn[2], cf[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      z[u] = zr[pc[u]];
      zn[u] = zr[sp[u] >= 0 ? sp[u] : pc[u]];
      cf[u] = coefp[pc[u]];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (p0 + 64 * u + lane < sg.p1 && gi[u] >= 0 && sp[u] >= 0) {
        T v[3] = {T(0), T(0), T(0)};
        phi<K, T>(v, a.p, z[u], zn[u], cf[u], prm);
        a.add(0, v[0]);
      }
    }
  }
}

// Problems with pair terms: one wave per row, lanes over the output groups and the pair
// positions of the row.
template <int P>
__global__ __launch_bounds__(256) void k_tiled_finalize_pairs(TiledProb tp, const typename Types<P>::T *__restrict__ partials,
                                                        const typename Types<P>::T *__restrict__ zbuf, int n,
                                                        typename Types<P>::T *__restrict__ out, int pstride) {
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
      switch (sg.kind) {
#define CUROB_PAIR_CASE(K) \
  case K: pair_terms<K, T>(tp, sg, zr, coefp, prm, lane, a); break;
        CUROB_PAIR_CASE(K_F7) CUROB_PAIR_CASE(K_GRIEROSEN) CUROB_PAIR_CASE(K_ROSENBROCK) CUROB_PAIR_CASE(K_F6)
#undef CUROB_PAIR_CASE
        default: break;
      }
#pragma unroll
      for (int sh = 1; sh < 64; sh <<= 1) {
        const T so = __shfl_xor(a.s[0], sh, 64);
        const T co = __shfl_xor(a.c[0], sh, 64);
        acc_merge(a, 0, so, co);
      }
    } else {
      // the segment's output groups in parallel over the lanes, then a butterfly merge
      for (int g0 = sg.g0; g0 < sg.g1; g0 += 64) {
        const int g = g0 + lane;
        if (g < sg.g1) {
          const T *src = partials + (static_cast<size_t>(g) * pstride + row) * kPartialSlots;
          T v[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) v[k] = src[k];
#pragma unroll
          for (int k = 0; k < 3; ++k) acc_merge(a, k, v[2 * k], v[2 * k + 1]);
          a.p *= v[6];
        }
      }
#pragma unroll
      for (int sh = 1; sh < 64; sh <<= 1) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const T so = __shfl_xor(a.s[k], sh, 64);
          const T co = __shfl_xor(a.c[k], sh, 64);
          acc_merge(a, k, so, co);
        }
        a.p *= __shfl_xor(a.p, sh, 64);
      }
    }
    if (lane == 0) {
      T s[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) s[k] = a.get_minus(k, sg.padc[k]);
      F += finalize_any<T>(sg.kind, s, a.p, sg.n);
    }
  }
  if (lane == 0) out[row] = F + T(tp.bias);
}

// Rows of one pack workgroup: the largest power of two <= 16 whose rows and position tables
// fit a quarter of the LDS (four workgroups per CU overlap their load and store phases), or
// the largest that fits the whole budget; 0 when even one row does not fit.
template <int P>
inline int pack_rows(const TiledProb &tp, int SX) {
  const int esz = P == PATH_F64 ? 8 : 4;
  const int fixed = round16(tp.Dp * 4) + round16(tp.D * esz);
  for (int R = 16; R >= 1; R >>= 1)
    if (fixed + R * SX * esz <= kMaxLdsBytes / 4) return R;
  for (int R = 16; R >= 1; R >>= 1)
    if (fixed + R * SX * esz <= kPackLdsBytes) return R;
  return 0;
}

// LDS row stride of the pack kernel (elements): >= D, a multiple of the vector width, and an
// odd multiple of 4 banks from row to row, so the 16 rows of a tile hit distinct banks.
template <int P>
inline int pack_stride(int D) {
  int sx = D;
  if constexpr (P == PATH_F64) {
    while (sx % 4 != 2) ++sx;  // 2 banks per element: 2 sx = 4 (mod 8)
  } else {
    while (sx % 8 != 4) ++sx;  // sx = 4 (mod 8)
  }
  return sx;
}

// pack, GEMM + formula, finalize for rows [0, n) of one path; the scratch holds `cap` rows
// (n <= cap, cap a multiple of the GEMM's row tile): the partial sums of output group g start
// at row g * cap, the pack and z buffers hold cap rows
template <int P, int... Ks>
hipError_t launch_tiled_path(int kind_hint, const TiledProb &tp, const void *x, void *out, int n, int cap,
                             void *partials, void *zbuf, void *pack, hipStream_t st, std::integer_sequence<int, Ks...>) {
  static const void *const gemm[] = {reinterpret_cast<const void *>(&k_tiled_gemm<P, Ks>)...};
  const void *fn = (kind_hint >= 0 && kind_hint < K_COUNT) ? gemm[kind_hint]
                                                           : reinterpret_cast<const void *>(&k_tiled_gemm<P, -1>);
  if (n > cap || cap % kTileRows != 0) return hipErrorInvalidValue;
  if (tp.rowwise) {
    if (kind_hint < 0 || kind_hint >= K_COUNT) return hipErrorInvalidValue;
    static const void *const rowwise[] = {reinterpret_cast<const void *>(&k_rowwise<P, Ks>)...};
    TiledProb arg = tp;
    const void *xa = x;
    void *oa = out;
    int na = n;
    void *args[] = {&arg, &xa, &na, &oa};
    return hipLaunchKernel(rowwise[kind_hint], dim3((n + 3) / 4), dim3(256), args, 0, st);
  }
  const int SX = pack_stride<P>(tp.D);
  const int R = pack_rows<P>(tp, SX);
  if (R == 0) return hipErrorInvalidValue;
  const int esz = P == PATH_F64 ? 8 : 4;
  const int lds = round16(tp.Dp * 4) + round16(tp.D * esz) + R * SX * esz;
  const void *pk = reinterpret_cast<const void *>(&k_tiled_pack<P>);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(pk, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
  }
  const int tiles = (n + kTileRows - 1) / kTileRows;  // the GEMM reads whole row tiles
  TiledProb arg = tp;
  const void *xa = x;
  void *pa = partials, *za = zbuf, *oa = out;
  unsigned char *pka = static_cast<unsigned char *>(pack);
  const unsigned char *pkc = pka;
  int na = n, Ra = R, SXa = SX;
  int va = ((tp.D * esz) % 16 == 0 && (reinterpret_cast<uintptr_t>(x) % 16) == 0) ? 1 : 0;
  void *pargs[] = {&arg, &xa, &na, &Ra, &SXa, &va, &pka};
  hipError_t e = hipLaunchKernel(pk, dim3(tiles * kTileRows / R), dim3(256), pargs, static_cast<size_t>(lds), st);
  if (e != hipSuccess) return e;
  int ta = tiles, ca = cap;
  void *gargs[] = {&arg, &pkc, &na, &ta, &pa, &za, &ca};
  const int rounds = (tiles + kNumXcd - 1) / kNumXcd;
  e = hipLaunchKernel(fn, dim3(tp.ngroups * rounds * kNumXcd), dim3(kGemmThreads), gargs, 0, st);
  if (e != hipSuccess) return e;
  void *fargs[] = {&arg, &pa, &za, &na, &oa, &ca};
  if (tp.any_pairwise)
    return hipLaunchKernel(reinterpret_cast<const void *>(&k_tiled_finalize_pairs<P>), dim3((n + 3) / 4), dim3(256),
                           fargs, 0, st);
  return hipLaunchKernel(reinterpret_cast<const void *>(&k_tiled_finalize<P>), dim3((n + 255) / 256), dim3(256), fargs,
                         0, st);
}

}  // namespace tiled

}  // namespace curob
