// eval_resident.h -- fused evaluation kernel for basic functions of dimension <= 128.
//
// Each wave evaluates 16 candidate rows per iteration and loops over row groups (grid-stride):
//   1. stage   the rows' x (contiguous in HBM) reach the wave's LDS slice through
//              bounds-checked buffer loads issued one iteration ahead, so that HBM traffic
//              overlaps everything below.  Rotated non-pairwise problems on the split paths load
//              straight into the slice (buffer loads that write LDS, issued as soon as the
//              gather has read the previous group); the others hold the rows in registers and
//              store them (the FP32/FP64-MFMA paths store y = x - o_hi, the split paths store x
//              and subtract o_hi in the gather);
//   2. rotate  Z^T = (s Qp) Y^T on the matrix cores over the nonzero tiles of the packed
//              block-diagonal rotation (Sec. 1.2: three random variable groups, one orthonormal
//              block each).  The B operand is gathered from LDS in group order; on the split
//              paths each y is cut into bf16 terms and the products accumulate in FP32;
//   3. phi     z = acc + c' and the formula, straight from the accumulator fragment (pairwise
//              families first exchange z through LDS to reach z_{i+1}); padded positions are
//              laid out so that they add exactly known constants, removed at the end;
//   4. reduce  groups of four terms summed plainly, then Kahan-compensated per lane, a two-step
//              cross-lane combine, finalise, store.
// The rotation tiles and per-position tables sit in LDS once per workgroup.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

#include "devprob.h"
#include "formulas.h"
#include "kernels.h"

namespace curob {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <int P>
struct PathT {
  using T = float;
  using V = f32x4;  // one 16-byte load
  using Acc4 = f32x4;
};
template <>
struct PathT<PATH_F64> {
  using T = double;
  using V = f64x2;
  using Acc4 = f64x4;
};

// Packed position held in accumulator element e of m-tile m by lane group q (= lane / 16).
// BF16 16x16x32 and FP32 16x16x4 place output row 4q+e in element e; FP64 16x16x4 places
// output row 4e+q there.  Unrotated problems use the first layout on every path.
template <int P, int ROT>
__device__ __forceinline__ int frag_pos(int m, int q, int e) {
  if constexpr (P == PATH_F64 && ROT) return 16 * m + 4 * e + q;
  else return 16 * m + 4 * q + e;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Copies the problem's table image (bytes, a multiple of 16, laid out as the fixed part of
// the LDS carve) to the start of LDS: each thread issues the loads of up to four 16-byte words
// (clamped indices, no branch around a load) before storing them, one round trip per round.
__device__ __forceinline__ void copy_image(unsigned char *dst, const void *src, int bytes) {
  const int4 *s = reinterpret_cast<const int4 *>(src);
  int4 *d = reinterpret_cast<int4 *>(dst);
  const int n = bytes >> 4;
  for (int base = threadIdx.x; base < n; base += 4 * blockDim.x) {
    int4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = base + u * blockDim.x;
      v[u] = s[i < n ? i : n - 1];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = base + u * blockDim.x;
      if (i < n) d[i] = v[u];
    }
  }
}

// Buffer resource over rows [row0, n) of x: loads past the end return zeros instead of
// faulting, so the last, partial row group needs no per-lane predicate.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rows_rsrc(const T *x, int row0, int n, int D) {
  const long long bytes = static_cast<long long>(n - row0) * D * static_cast<long long>(sizeof(T));
  const int nb = bytes > 0x7ffffff0LL ? 0x7ffffff0 : static_cast<int>(bytes);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(x + static_cast<size_t>(row0) * D), (short)0, nb,
                                           0x00020000);
}

// Loads a row group straight into the wave's LDS slice (buffer loads that write LDS; no
// register holds the data): row r of the group, 4D bytes from byte 4rD of the resource, lands at
// Y + rS.  16-byte loads when every row starts 16-byte aligned in memory, 4-byte loads
// otherwise; lanes past a row's length are masked off, so nothing is written past column D - 1.
// The wave must wait for the vector-memory counter before reading the slice.
__device__ __forceinline__ void load_rows_direct(__amdgpu_buffer_rsrc_t rs, int D, int S, float *Y, bool wide,
                                                 int lane) {
  typedef __attribute__((address_space(3))) void *lds_ptr;
  if (wide) {
    if (lane < (D >> 2)) {
#pragma unroll
      for (int r = 0; r < kRowsPerBlock; ++r)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_ptr)(Y + r * S), 16, lane * 16, r * 4 * D, 0, 0);
    }
  } else {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (lane + 64 * h < D) {
#pragma unroll
        for (int r = 0; r < kRowsPerBlock; ++r)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_ptr)(Y + r * S + 64 * h), 4, (lane + 64 * h) * 4, r * 4 * D,
                                                   0, 0);
      }
    }
  }
}

// s_waitcnt operands (gfx9 encoding): wait for every vector-memory operation, or for every
// LDS operation, leaving the other counters free.
constexpr int kWaitVmem = 0x3F70;
constexpr int kWaitLds = 0xC07F;

// Registers holding a wave's rows between their load and their staging: 16-byte loads when
// the dimension is a multiple of the vector width (VEC), element loads otherwise.
template <int P, int VEC>
struct XTile {
  using T = typename PathT<P>::T;
  using V = typename PathT<P>::V;
  static constexpr int ROWS = kRowsPerBlock * blocks_of(P);
  static constexpr int NV = VEC ? 16 / static_cast<int>(sizeof(T)) : 1;  // elements per load
  static constexpr int CMAX = ROWS * 16 * kMaxMT / (64 * NV);            // loads per lane, D <= 128
  using L = typename std::conditional<VEC, V, T>::type;
  L v[CMAX];

  // registers past the row group's loads stay zero (raw staging stores them to the spill row)
  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int t = 0; t < CMAX; ++t) v[t] = L{};
  }

  __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, int nload, int lane) {
#pragma unroll
    for (int t = 0; t < CMAX; ++t) {
      if (t < nload) {
        const int off = (lane + 64 * t) * NV * static_cast<int>(sizeof(T));
        if constexpr (VEC) {
          v[t] = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
        } else if constexpr (sizeof(T) == 8) {
          v[t] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
        } else {
          v[t] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
        }
      }
    }
  }

  // stage with the shift vectors read first, all together; stores past nload reach the spill
  // row only (the registers beyond the row group's loads hold values never used)
  __device__ __forceinline__ void stage_batched(int D, int S, T *Y, const T *oh, int lane) const {
    const int e0 = lane * NV;
    constexpr int step = 64 * NV;
    const int dr = step / D, dj = step - dr * D;
    L o[CMAX];
    {
      int jj = e0 % D;
#pragma unroll
      for (int t = 0; t < CMAX; ++t) {
        if constexpr (VEC) o[t] = *reinterpret_cast<const V *>(oh + jj);
        else o[t] = oh[jj];
        jj += dj;
        jj = jj >= D ? jj - D : jj;
      }
    }
    int rr = e0 / D, jj = e0 - rr * D;
#pragma unroll
    for (int t = 0; t < CMAX; ++t) {
      const int ra = rr < ROWS ? rr : ROWS;
      if constexpr (VEC) *reinterpret_cast<V *>(Y + ra * S + jj) = v[t] - o[t];
      else Y[ra * S + jj] = v[t] - o[t];
      jj += dj;
      rr += dr;
      if (jj >= D) {
        jj -= D;
        ++rr;
      }
    }
  }

  // Y[r][j] = x[r][j] - o_hi[j] (RAW: x[r][j]; the split paths subtract o_hi later, in packed
  // order) for the wave's rows; elements past the last row land in the spill row ROWS of the
  // slice.  RAW stores need neither a shift read nor a guard: registers past nload hold zeros
  // and only reach the spill row.
  template <bool RAW>
  __device__ __forceinline__ void stage(int nload, int D, int S, T *Y, const T *oh, int lane) const {
    if constexpr (!RAW && sizeof(T) == 8) {
      // FP64 (two waves per SIMD, registers to spare): every shift read is issued before the
      // first subtraction, one LDS round trip instead of one per load
      stage_batched(D, S, Y, oh, lane);
      return;
    }
    const int e0 = lane * NV;
    int rr = e0 / D, jj = e0 - rr * D;
    constexpr int step = 64 * NV;
    const int dr = step / D, dj = step - dr * D;
#pragma unroll
    for (int t = 0; t < CMAX; ++t) {
      if (RAW || t < nload) {
        const int ra = rr < ROWS ? rr : ROWS;
        if constexpr (RAW) {
          if constexpr (VEC) *reinterpret_cast<V *>(Y + ra * S + jj) = v[t];
          else Y[ra * S + jj] = v[t];
        } else if constexpr (VEC) {
          *reinterpret_cast<V *>(Y + ra * S + jj) = v[t] - *reinterpret_cast<const V *>(oh + jj);
        } else {
          Y[ra * S + jj] = v[t] - oh[jj];
        }
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

// Per-path operand types of the rotation: B fragments for every k-tile stay in registers
// ("B stationary") while the m-tiles stream past them.
template <int P>
struct RotOps;
template <>
struct RotOps<PATH_SPLIT> {
  static constexpr int KTMAX = 16 * kMaxMT / 32;  // k-tiles of 32 for dimension <= 128
  static constexpr int NTERM = 2;
  using Frag = bf16x8;
};
template <>
struct RotOps<PATH_SPLIT6> {
  static constexpr int KTMAX = 16 * kMaxMT / 32;
  static constexpr int NTERM = 3;
  using Frag = bf16x8;
};
template <>
struct RotOps<PATH_F32> {
  static constexpr int KTMAX = 16 * kMaxMT / 4;  // k-tiles of 4
  static constexpr int NTERM = 1;
  using Frag = float;
};
template <>
struct RotOps<PATH_F64> {
  static constexpr int KTMAX = 16 * kMaxMT / 4;
  static constexpr int NTERM = 1;
  using Frag = double;
};

// Cuts two gathered elements y (positions e, e + 1 of k-tile kt) into the split path's bf16
// terms: y - hi and the next residual are exact in FP32.
template <int P>
__device__ __forceinline__ void cut_terms(typename RotOps<P>::Frag (&bf)[RotOps<P>::NTERM][blocks_of(P)][RotOps<P>::KTMAX],
                                          int b, int kt, int e, f32x2 y) {
  const bf16x2 h = __builtin_convertvector(y, bf16x2);
  const f32x2 r1 = y - __builtin_convertvector(h, f32x2);
  bf[0][b][kt][e] = h[0];
  bf[0][b][kt][e + 1] = h[1];
  if constexpr (RotOps<P>::NTERM == 3) {
    const bf16x2 m = __builtin_convertvector(r1, bf16x2);
    const bf16x2 l = __builtin_convertvector(r1 - __builtin_convertvector(m, f32x2), bf16x2);
    bf[1][b][kt][e] = m[0];
    bf[1][b][kt][e + 1] = m[1];
    bf[2][b][kt][e] = l[0];
    bf[2][b][kt][e + 1] = l[1];
  } else {
    const bf16x2 l = __builtin_convertvector(r1, bf16x2);
    bf[1][b][kt][e] = l[0];
    bf[1][b][kt][e + 1] = l[1];
  }
}

// Gathers this lane's B operand of every k-tile and column block from the staged rows (packed
// order via the byte offsets s_goff) and, on the split paths, subtracts o_hi (s_ohp, packed
// order) and cuts each y into bf16 terms.  Yb: row r of column block 0.
template <int P>
__device__ __forceinline__ void gather_b(typename RotOps<P>::Frag (&bf)[RotOps<P>::NTERM][blocks_of(P)][RotOps<P>::KTMAX],
                                         int KT, const uint16_t *s_goff, const unsigned char *Yb, int bstride,
                                         int q, const float *s_ohp) {
  using R = RotOps<P>;
  constexpr int NB = blocks_of(P);
#pragma unroll
  for (int kt = 0; kt < R::KTMAX; ++kt) {
    if (kt < KT) {
      if constexpr (is_split(P)) {
        const uint4 idx = *reinterpret_cast<const uint4 *>(s_goff + kt * 32 + q * 8);
        const uint32_t iw[4] = {idx.x, idx.y, idx.z, idx.w};
        // the rows hold x: y = x - o_hi with o_hi in packed order (one rounding, as when staged)
        const f32x4 oa = *reinterpret_cast<const f32x4 *>(s_ohp + kt * 32 + q * 8);
        const f32x4 ob = *reinterpret_cast<const f32x4 *>(s_ohp + kt * 32 + q * 8 + 4);
        const float ov[8] = {oa[0], oa[1], oa[2], oa[3], ob[0], ob[1], ob[2], ob[3]};
        // the k-tile's eight element reads are issued together, then the cuts
        float xv[NB][8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const uint32_t oe = (e & 1) ? iw[e >> 1] >> 16 : iw[e >> 1] & 0xFFFFu;
#pragma unroll
          for (int b = 0; b < NB; ++b) xv[b][e] = *reinterpret_cast<const float *>(Yb + b * bstride + oe);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
          // two elements at a time: one packed conversion per term for the pair
          const f32x2 oo = {ov[e], ov[e + 1]};
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const f32x2 y = f32x2{xv[b][e], xv[b][e + 1]} - oo;
            cut_terms<P>(bf, b, kt, e, y);
          }
        }
      } else {
        const uint32_t off = s_goff[kt * 4 + q];
#pragma unroll
        for (int b = 0; b < NB; ++b)
          bf[0][b][kt] = *reinterpret_cast<const typename R::Frag *>(Yb + b * bstride + off);
      }
    }
  }
}

// The same gather on a split path from addresses computed once per launch: ga holds the LDS
// byte address (from lds) of every element this lane reads, 8 per k-tile, so a row group costs
// no offset-table reads and no address arithmetic (one column block).
template <int P>
__device__ __forceinline__ void gather_pre(typename RotOps<P>::Frag (&bf)[RotOps<P>::NTERM][blocks_of(P)][RotOps<P>::KTMAX],
                                           int KT, const uint32_t (&ga)[RotOps<P>::KTMAX * 8], const unsigned char *lds,
                                           int q, const float *s_ohp) {
  using R = RotOps<P>;
#pragma unroll
  for (int kt = 0; kt < R::KTMAX; ++kt) {
    if (kt < KT) {
      const f32x4 oa = *reinterpret_cast<const f32x4 *>(s_ohp + kt * 32 + q * 8);
      const f32x4 ob = *reinterpret_cast<const f32x4 *>(s_ohp + kt * 32 + q * 8 + 4);
      // the k-tile's eight element reads are issued together, then the cuts (left to itself the
      // compiler waits for each pair of reads before its cut)
      float xv[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) xv[e] = *reinterpret_cast<const float *>(lds + ga[kt * 8 + e]);
      __builtin_amdgcn_sched_barrier(0);
      const float ov[8] = {oa[0], oa[1], oa[2], oa[3], ob[0], ob[1], ob[2], ob[3]};
#pragma unroll
      for (int e = 0; e < 8; e += 2) {
        const f32x2 oo = {ov[e], ov[e + 1]};
        const f32x2 y = f32x2{xv[e], xv[e + 1]} - oo;
        cut_terms<P>(bf, 0, kt, e, y);
      }
    }
  }
}

// One m-tile of Z^T = (s Qp) Y^T for all column blocks on the FP32 and FP64 MFMA paths (the
// split paths use mtile_fixed): acc[b] element e is packed position frag_pos(m, q, e).
// mi = (first k-tile, last k-tile, first tile index) of m-tile m.
template <int P>
__device__ __forceinline__ void mtile(typename PathT<P>::Acc4 (&acc)[blocks_of(P)], int4 mi,
                                      const typename RotOps<P>::Frag (&bf)[RotOps<P>::NTERM][blocks_of(P)][RotOps<P>::KTMAX],
                                      const unsigned char *s_q, int lane) {
  using R = RotOps<P>;
  using Acc4 = typename PathT<P>::Acc4;
  constexpr int NB = blocks_of(P);
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = Acc4{0, 0, 0, 0};
#pragma unroll
  for (int kt = 0; kt < R::KTMAX; ++kt) {
    if (kt >= mi.x && kt <= mi.y) {
      const int t = mi.z + kt - mi.x;
      {
        const auto a = reinterpret_cast<const typename R::Frag *>(s_q)[t * 64 + lane];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          if constexpr (P == PATH_F64)
            acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bf[0][b][kt], acc[b], 0, 0, 0);
          else
            acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bf[0][b][kt], acc[b], 0, 0, 0);
        }
      }
    }
  }
}

// One m-tile on the split paths for a k range fixed at compile time (k-tiles KX .. KX+NK-1):
// each k-tile's rotation fragments are requested from LDS before the previous k-tile's products
// are issued (held apart by a scheduling barrier; left to itself the compiler reuses one register
// set and waits for every read next to its product), and the products run with no branch
// between them.
template <int P, int KX, int NK>
__device__ __forceinline__ void mtile_fixed(typename PathT<P>::Acc4 (&acc)[blocks_of(P)], int t0,
                                            const bf16x8 (&bf)[RotOps<P>::NTERM][blocks_of(P)][RotOps<P>::KTMAX],
                                            const unsigned char *s_q, int lane) {
  constexpr int NT = RotOps<P>::NTERM;
  constexpr int NB = blocks_of(P);
  const bf16x8 *qf = reinterpret_cast<const bf16x8 *>(s_q) + t0 * (64 * NT) + lane;
  bf16x8 qa[NK][NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) qa[0][u] = qf[u * 64];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = f32x4{0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < NK; ++j) {
    const int kt = KX + j;
    if (j + 1 < NK) {
#pragma unroll
      for (int u = 0; u < NT; ++u) qa[j + 1][u] = qf[((j + 1) * NT + u) * 64];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if constexpr (NT == 3) {
        // the six products of total order <= 2 in the 2^-8 splitting, smallest first
        acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(qa[j][2], bf[0][b][kt], acc[b], 0, 0, 0);
        acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(qa[j][1], bf[1][b][kt], acc[b], 0, 0, 0);
        acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(qa[j][0], bf[2][b][kt], acc[b], 0, 0, 0);
        acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(qa[j][1], bf[0][b][kt], acc[b], 0, 0, 0);
        acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(qa[j][0], bf[1][b][kt], acc[b], 0, 0, 0);
        acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(qa[j][0], bf[0][b][kt], acc[b], 0, 0, 0);
      } else {
        acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(qa[j][1], bf[0][b][kt], acc[b], 0, 0, 0);
        acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(qa[j][0], bf[1][b][kt], acc[b], 0, 0, 0);
        acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(qa[j][0], bf[0][b][kt], acc[b], 0, 0, 0);
      }
    }
  }
}

// Calls f(std::integral_constant<int, C>) for the k-range code C = 4 * first k-tile + (k-tiles - 1)
// of an m-tile (split paths: at most four k-tiles of 32).
template <typename F>
__device__ __forceinline__ void dispatch_krange(int code, F &&f) {
  switch (code) {
#define CUROB_KCASE(C) \
  case C:              \
    f(std::integral_constant<int, C>{}); \
    break;
    CUROB_KCASE(0) CUROB_KCASE(1) CUROB_KCASE(2) CUROB_KCASE(3) CUROB_KCASE(4) CUROB_KCASE(5)
    CUROB_KCASE(6) CUROB_KCASE(8) CUROB_KCASE(9) CUROB_KCASE(12)
#undef CUROB_KCASE
    default:
      break;
  }
}

// One m-tile on the 4-wide paths (FP32 and FP64 MFMA) with B read from the staged rows inside
// a runtime loop over the m-tile's k range: no per-k-tile branches over the full 32-tile
// range and no register-resident B, so more waves fit.  Two accumulators halve the dependent
// chain of MFMAs.
template <int P>
__device__ __forceinline__ void mtile_stream(typename PathT<P>::Acc4 (&acc)[1], int4 mi, const uint16_t *s_goff,
                                             const unsigned char *Yb, const unsigned char *s_q, int lane, int q) {
  using Frag = typename RotOps<P>::Frag;
  using Acc4 = typename PathT<P>::Acc4;
  Acc4 a0 = Acc4{0, 0, 0, 0}, a1 = Acc4{0, 0, 0, 0};
  const Frag *qa = reinterpret_cast<const Frag *>(s_q) + (mi.z - mi.x) * 64 + lane;
  int kt = mi.x;
  for (; kt < mi.y; kt += 2) {
    const Frag b0 = *reinterpret_cast<const Frag *>(Yb + s_goff[kt * 4 + q]);
    const Frag b1 = *reinterpret_cast<const Frag *>(Yb + s_goff[kt * 4 + 4 + q]);
    if constexpr (P == PATH_F64) {
      a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[kt * 64], b0, a0, 0, 0, 0);
      a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[kt * 64 + 64], b1, a1, 0, 0, 0);
    } else {
      a0 = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[kt * 64], b0, a0, 0, 0, 0);
      a1 = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[kt * 64 + 64], b1, a1, 0, 0, 0);
    }
  }
  if (kt == mi.y) {
    const Frag b0 = *reinterpret_cast<const Frag *>(Yb + s_goff[kt * 4 + q]);
    if constexpr (P == PATH_F64)
      a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[kt * 64], b0, a0, 0, 0, 0);
    else
      a0 = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[kt * 64], b0, a0, 0, 0, 0);
  }
  acc[0] = a0 + a1;
}

// The four packed positions frag_pos(m, q, 0..3) of a row as one vector from LDS (unrotated
// layout: consecutive, 16-byte aligned because S and 16 m + 4 q are multiples of 4).
template <typename T>
__device__ __forceinline__ void read4(T (&v)[4], const T *row, int p0) {
  if constexpr (sizeof(T) == 4) {
    const f32x4 t = *reinterpret_cast<const f32x4 *>(row + p0);
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = t[e];
  } else {
    const f64x2 t0 = *reinterpret_cast<const f64x2 *>(row + p0);
    const f64x2 t1 = *reinterpret_cast<const f64x2 *>(row + p0 + 2);
    v[0] = t0[0];
    v[1] = t0[1];
    v[2] = t1[0];
    v[3] = t1[1];
  }
}

// Evaluates row groups g, g + gstride, ... < gend of one problem with the calling wave
// (the workgroup's waves share the problem's LDS tables).  setup: copy the tables and clear
// the slices' padding columns first (every wave of the workgroup must take part).
template <int P, int KIND, int ROT, int VEC>
__device__ __forceinline__ void resident_eval(const DevProb &pb, const typename PathT<P>::T *__restrict__ x,
                                              typename PathT<P>::T *__restrict__ out, int n, int g, int gend,
                                              int gstride, int nwaves, int wave, bool setup, unsigned char *smem) {
  using T = typename PathT<P>::T;
  using Acc4 = typename PathT<P>::Acc4;
  using Tile = XTile<P, VEC>;
  using KT_ = KindTraits<KIND>;
  using R = RotOps<P>;
  constexpr int NB = blocks_of(P);
  constexpr int ROWS = Tile::ROWS;
  const LdsLayout L = lds_layout(P, pb, nwaves);
  const unsigned char *s_q = smem + L.q;
  const uint16_t *s_goff = reinterpret_cast<const uint16_t *>(smem + L.goff);
  const T *s_oh = reinterpret_cast<const T *>(smem + L.oh);
  const T *s_cz = reinterpret_cast<const T *>(smem + L.cz);
  const T *s_coef = reinterpret_cast<const T *>(smem + L.coef);
  const int16_t *s_succ = reinterpret_cast<const int16_t *>(smem + L.succ);

  const int D = pb.D, S = pb.S, MT = pb.MT;
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, q = lane >> 4;
  const int nload = (ROWS * D + 64 * Tile::NV - 1) / (64 * Tile::NV);

  // rows loaded straight into the slice, or staged through registers
  constexpr bool DIRECT = direct_rows(P, ROT, KIND);
  T *Y = reinterpret_cast<T *>(smem + L.y + wave * L.slice_bytes);
  // (direct) every row starts 16-byte aligned in memory: D a multiple of 4 and x aligned
  const bool wide = (D & 3) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;
  // staged: the first row group's loads go out before the tables are copied.  Direct: after
  // the copy (in a batch the LDS may still hold another problem's tables until the barrier)
  Tile xt;
  if constexpr (!DIRECT) {
    if constexpr (is_split(P) || P == PATH_F64) xt.clear();
    if (g < gend) xt.load(rows_rsrc(x, g * ROWS, n, D), nload, lane);
  }
  if (setup) {
    // every table (the k ranges included: read from global memory inside the loop, their
    // vector-memory wait would also wait for the next row group's prefetch) in one pass
    copy_image(smem, pb.image, pb.image_bytes);
    // columns D..S-1 of every row are zero: the gather's padding slot and the unrotated read-out
    for (int i = lane; i < ROWS * (S - D); i += 64) Y[(i / (S - D)) * S + D + i % (S - D)] = T(0);
    __syncthreads();
  }
  if constexpr (DIRECT) {
    if (g < gend) load_rows_direct(rows_rsrc(x, g * ROWS, n, D), D, S, reinterpret_cast<float *>(Y), wide, lane);
  }

  const T scale = T(pb.scale);
  const T prm = kind_param<KIND, T>(pb.Df, pb.kparam);
  const unsigned char *Yb = reinterpret_cast<const unsigned char *>(Y + r * S);
  const int bstride = kRowsPerBlock * S * static_cast<int>(sizeof(T));
  const int4 *s_mtab = reinterpret_cast<const int4 *>(smem + L.mtab);

  // three-product direct path: the gather addresses are fixed for the launch and fit the
  // registers the staged rows would have used (the six-product path has no room for them)
  constexpr bool PRE = DIRECT && P == PATH_SPLIT;
  uint32_t ga[RotOps<P>::KTMAX * 8];
  if constexpr (PRE) {
    const uint32_t ybase = static_cast<uint32_t>(reinterpret_cast<const unsigned char *>(Y + r * S) - smem);
#pragma unroll
    for (int kt = 0; kt < RotOps<P>::KTMAX; ++kt) {
      const uint4 idx = *reinterpret_cast<const uint4 *>(s_goff + (kt < pb.KT ? kt : 0) * 32 + q * 8);
      const uint32_t iw[4] = {idx.x, idx.y, idx.z, idx.w};
#pragma unroll
      for (int e = 0; e < 8; e += 2) {
        ga[kt * 8 + e] = ybase + (iw[e >> 1] & 0xFFFFu);
        ga[kt * 8 + e + 1] = ybase + (iw[e >> 1] >> 16);
      }
    }
  }
  // (direct) the result of the previous row group, stored once the next group's rows have
  // been requested: its store then never delays the wait for those rows
  T pend = T(0);
  int prow = n;
  for (; g < gend; g += gstride) {
    const int row0 = g * ROWS;
    const int gn = g + gstride;
    if constexpr (DIRECT) {
      // the row group's loads, issued one iteration earlier, have landed in the slice
      __builtin_amdgcn_s_waitcnt(kWaitVmem);
      wave_sync();
      // the gather leads to the group's first products: it runs at raised priority too
      __builtin_amdgcn_s_setprio(1);
    } else {
      wave_sync();
      xt.template stage<is_split(P)>(nload, D, S, Y, s_oh, lane);
      // the next row group's loads are in flight during everything below
      if (gn < gend) xt.load(rows_rsrc(x, gn * ROWS, n, D), nload, lane);
      wave_sync();
    }

    // 4-wide paths without pairwise z exchange read B from the rows in the m-tile loop
    constexpr bool SB = ROT && !is_split(P) && !KT_::pairwise && NB == 1;
    typename R::Frag bf[R::NTERM][NB][R::KTMAX];
    if constexpr (ROT && !SB) {
      if constexpr (PRE) gather_pre<P>(bf, pb.KT, ga, smem, q, reinterpret_cast<const float *>(s_oh));
      else gather_b<P>(bf, pb.KT, s_goff, Yb, bstride, q, reinterpret_cast<const float *>(s_oh));
      if constexpr (KT_::pairwise) wave_sync();  // the rows are overwritten with z below
    }
    if constexpr (DIRECT) {
      // the gather's reads of the slice are complete before the next group's rows overwrite it
      __builtin_amdgcn_s_waitcnt(kWaitLds);
      wave_sync();
      __builtin_amdgcn_s_setprio(0);
      if (gn < gend) load_rows_direct(rows_rsrc(x, gn * ROWS, n, D), D, S, reinterpret_cast<float *>(Y), wide, lane);
      if (q == 0 && prow < n) out[prow] = pend;
    }
    auto rotate_m = [&](Acc4 (&acc)[NB], int mm) {
      const int4 mv = s_mtab[mm];
      const int4 mi = make_int4(__builtin_amdgcn_readfirstlane(mv.x), __builtin_amdgcn_readfirstlane(mv.y),
                                __builtin_amdgcn_readfirstlane(mv.z), 0);
      if constexpr (SB) mtile_stream<P>(acc, mi, s_goff, Yb, s_q, lane, q);
      else if constexpr (!is_split(P)) mtile<P>(acc, mi, bf, s_q, lane);
    };
    // split paths: the m-tile's k range selects a branch-free product sequence
    constexpr bool FIX = ROT && is_split(P);
    auto rotate_fix = [&](Acc4 (&acc)[NB], int4 mv) {
      if constexpr (FIX) {
        const int code = __builtin_amdgcn_readfirstlane(mv.w);
        const int t0 = __builtin_amdgcn_readfirstlane(mv.z);
        // the wave issues its products at raised priority, so the matrix core gets them ahead
        // of other waves' formula work on the SIMD
        __builtin_amdgcn_s_setprio(1);
        dispatch_krange(code, [&](auto c) {
          constexpr int C = decltype(c)::value;
          mtile_fixed<P, C / 4, C % 4 + 1>(acc, t0, bf, s_q, lane);
        });
        __builtin_amdgcn_s_setprio(0);
      }
    };

    Acc<T> a[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) a[b].init();

    // rotated: the MFMAs of m-tile m + 1 are issued before the formula work of m-tile m, so
    // the matrix cores and the vector ALUs overlap within the wave
    // (not on the FP64 path, whose doubled accumulators would not fit the registers)
    constexpr bool PIPE = P != PATH_F64;
    Acc4 acc_cur[NB], acc_nxt[NB];
    int4 mv_next = make_int4(0, 0, 0, 0);  // k range of m-tile m + 1, read one m-tile ahead
    if constexpr (FIX) {
      rotate_fix(acc_cur, s_mtab[0]);
      mv_next = s_mtab[MT > 1 ? 1 : 0];
    } else if constexpr (ROT && PIPE) {
      rotate_m(acc_cur, 0);
    }
    for (int m = 0; m < MT; ++m) {
      T z[NB][4];
      // the m-tile's per-position tables are read before the next m-tile's products are
      // issued, so their LDS latency hides behind the MFMAs
      T c4[4], cf[4] = {T(0), T(0), T(0), T(0)};
      if constexpr (P == PATH_F64 && ROT) {
#pragma unroll
        for (int e = 0; e < 4; ++e) c4[e] = s_cz[frag_pos<P, ROT>(m, q, e)];
        if constexpr (KT_::needs_coef && !KT_::pairwise) {
#pragma unroll
          for (int e = 0; e < 4; ++e) cf[e] = s_coef[frag_pos<P, ROT>(m, q, e)];
        }
      } else {
        read4(c4, s_cz, 16 * m + 4 * q);
        if constexpr (KT_::needs_coef && !KT_::pairwise) read4(cf, s_coef, 16 * m + 4 * q);
      }
      if constexpr (ROT) {
        if constexpr (FIX) {
          const int4 mv2 = s_mtab[m + 2 < MT ? m + 2 : MT - 1];
          if (m + 1 < MT) rotate_fix(acc_nxt, mv_next);
          mv_next = mv2;
        } else if constexpr (PIPE) {
          if (m + 1 < MT) rotate_m(acc_nxt, m + 1);
        } else {
          rotate_m(acc_cur, m);
        }
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int e = 0; e < 4; ++e) z[b][e] = T(acc_cur[b][e]) + c4[e];
        if constexpr (PIPE) {
#pragma unroll
          for (int b = 0; b < NB; ++b) acc_cur[b] = acc_nxt[b];
        }
      } else {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          T y4[4];
          read4(y4, Y + (b * kRowsPerBlock + r) * S, 16 * m + 4 * q);
          if constexpr (is_split(P)) {
            // raw rows: y = x - o_hi here (packed order is the original order when unrotated)
            T o4[4];
            read4(o4, s_oh, 16 * m + 4 * q);
#pragma unroll
            for (int e = 0; e < 4; ++e) y4[e] -= o4[e];
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) z[b][e] = scale * y4[e] + c4[e];
        }
      }
      if constexpr (KT_::pairwise) {
        // z goes back to the rows (packed order); the terms need the successors, read below
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int e = 0; e < 4; ++e) Y[(b * kRowsPerBlock + r) * S + frag_pos<P, ROT>(m, q, e)] = z[b][e];
      } else {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          T v[3] = {T(0), T(0), T(0)};
#pragma unroll
          for (int e = 0; e < 4; ++e) phi<KIND, T>(v, a[b].p, z[b][e], T(0), cf[e], prm);
#pragma unroll
          for (int k = 0; k < KT_::nsum; ++k) acc_add<KIND, T>(a[b], k, v[k]);
        }
      }
    }

    if constexpr (KT_::pairwise && P != PATH_F64) {
      // a lane's four positions of an m-tile are consecutive (16 m + 4 q + e): their successor
      // indices (one 8-byte read), own z (one 16-byte read) and the four successors' z are all
      // requested before the formula work, one LDS round trip per m-tile instead of one per
      // element
      typedef short i16x4 __attribute__((ext_vector_type(4)));
      wave_sync();
      for (int m = 0; m < MT; ++m) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const T *zr = Y + (b * kRowsPerBlock + r) * S;
          const int p0 = 16 * m + 4 * q;
          const i16x4 s4 = *reinterpret_cast<const i16x4 *>(s_succ + p0);
          const f32x4 own = *reinterpret_cast<const f32x4 *>(zr + p0);
          const int sp[4] = {s4[0], s4[1], s4[2], s4[3]};
          T nx[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) nx[e] = zr[sp[e] < 0 ? p0 + e : sp[e]];
          // keep the reads together ahead of the arithmetic
          __builtin_amdgcn_sched_barrier(0);
          T v = T(0);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            T w[3] = {T(0), T(0), T(0)};
            phi<KIND, T>(w, a[b].p, own[e], nx[e], T(0), prm);
            v += sp[e] < 0 ? T(0) : w[0];
          }
          acc_add<KIND, T>(a[b], 0, v);
        }
      }
    } else if constexpr (KT_::pairwise) {
      // FP64 rotated layout: a lane's positions 16 m + 4 e + q are not consecutive
      wave_sync();
      for (int m = 0; m < MT; ++m) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const T *zr = Y + (b * kRowsPerBlock + r) * S;
          T v[3] = {T(0), T(0), T(0)};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int p = frag_pos<P, ROT>(m, q, e);
            const int sp = s_succ[p];
            T w[3] = {T(0), T(0), T(0)};
            phi<KIND, T>(w, a[b].p, zr[p], zr[sp < 0 ? p : sp], T(0), prm);
            v[0] += sp < 0 ? T(0) : w[0];
          }
          acc_add<KIND, T>(a[b], 0, v[0]);
        }
      }
    }

#pragma unroll
    for (int b = 0; b < NB; ++b) {
      // combine the four lanes that hold the same row (lane, lane^16, lane^32, lane^48)
#pragma unroll
      for (int sh = 16; sh <= 32; sh <<= 1) {
#pragma unroll
        for (int k = 0; k < KT_::nsum; ++k) {
          const T so = __shfl_xor(a[b].s[k], sh, 64);
          const T co = __shfl_xor(a[b].c[k], sh, 64);
          acc_merge(a[b], k, so, co);
        }
        if constexpr (KT_::has_product) a[b].p *= __shfl_xor(a[b].p, sh, 64);
      }
      const int row = row0 + b * kRowsPerBlock + r;
      if constexpr (DIRECT) {
        T s[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) s[k] = a[b].get_minus(k, pb.padc[k]);
        pend = finalize<KIND, T>(s, a[b].p, pb.Df) + T(pb.bias);
        prow = row;
      } else if (q == 0 && row < n) {
        T s[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) s[k] = a[b].get_minus(k, pb.padc[k]);
        out[row] = finalize<KIND, T>(s, a[b].p, pb.Df) + T(pb.bias);
      }
    }
  }
  if constexpr (DIRECT) {
    if (q == 0 && prow < n) out[prow] = pend;
  }
}

template <int P, int KIND, int ROT, int VEC>
__global__ __launch_bounds__(64 * max_waves_of(P, direct_rows(P, ROT, KIND))) void k_eval_resident(DevProb pb, const typename PathT<P>::T *__restrict__ x,
                                                       typename PathT<P>::T *__restrict__ out, int n) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nwaves = blockDim.x >> 6;
  // wave-uniform values live in scalar registers: the row-group loop and the buffer
  // resources built from it stay scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  constexpr int ROWS = XTile<P, VEC>::ROWS;
  const int ngroups = (n + ROWS - 1) / ROWS;
  resident_eval<P, KIND, ROT, VEC>(pb, x, out, n, blockIdx.x * nwaves + wave, ngroups, gridDim.x * nwaves, nwaves,
                                   wave, true, smem);
}

// Kernel table of one path: index ((kind * 2) + rot) * 2 + vec.
template <int P, int... Ks>
const void *const *resident_table(std::integer_sequence<int, Ks...>) {
  static const void *const tab[] = {
      (reinterpret_cast<const void *>(&k_eval_resident<P, Ks / 4, (Ks / 2) % 2, Ks % 2>))...};
  return tab;
}

}  // namespace curob
