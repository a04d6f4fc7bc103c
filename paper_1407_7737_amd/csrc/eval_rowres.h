// eval_rowres.h -- fused evaluation for dimensions above the resident kernel's range on the
// split paths (basic functions and hybrids, Sec. 5), with the population rows resident in LDS.
//
// A workgroup of eight waves holds 16 * CB population rows in LDS (x as read, one row at a time
// with buffer loads that write LDS) and computes every output of the packed block-diagonal
// rotation for them:
//   - for each rotation block, each wave takes m-tiles (16 outputs) of the block, up to three at
//     a time, and walks the block's k steps: the B operand (y = x - o_hi of 8 packed positions
//     per lane, cut into bf16 terms) is gathered from the LDS rows once per step and feeds all
//     of the wave's m-tiles; the rotation tiles (A operand) stream from L2, two steps ahead;
//   - z = acc + c' then the formula's per-element terms go into the wave's compensated row
//     sums (formulas with pair terms instead write z to an LDS copy in packed order);
//   - row sums of all waves meet in LDS, in wave order, and wave 0 finalises each formula
//     segment of its rows; pair terms are summed from the LDS copy of z at the end.
// X is read from HBM once, nothing goes through scratch memory, and the result row is written
// directly.  Persistent grid: each workgroup walks row tiles with a stride of the grid.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

#include "devprob.h"
#include "formulas.h"
#include "kernels.h"
#include "tiled.h"

namespace curob {

namespace rowres {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
constexpr int kMW = 3;      // m-tiles of one block per wave pass (one B gather feeds them all)
constexpr int kSlots = 8;   // per (wave, row) partial: s0 c0 s1 c1 s2 c2 product pad

// LDS carve: packed-position tables, the rows, the z copy (pairwise), the per-wave partials.
struct Carve {
  int goff, ohp, rows, zc, red, total;
};
__host__ __device__ inline Carve carve(int Dp, int S, int CB, bool pairs) {
  Carve c;
  const int R = 16 * CB;
  c.goff = 0;
  c.ohp = round16(Dp * 2);
  c.rows = c.ohp + round16(Dp * 4);
  c.zc = c.rows + round16(R * S * 4);
  c.red = c.zc + (pairs ? round16(R * Dp * 4) : 0);
  c.total = c.red + kWaves * R * kSlots * 4;
  return c;
}

template <typename T>
__device__ __forceinline__ T finalize_kind(int kind, const T (&s)[3], T p, int n) {
  switch (kind) {
#define CUROB_RR_FIN(K) \
  case K: return finalize<K, T>(s, p, n);
    CUROB_RR_FIN(K_WSPHERE) CUROB_RR_FIN(K_POWERS) CUROB_RR_FIN(K_SHARPV) CUROB_RR_FIN(K_STEP)
    CUROB_RR_FIN(K_WEIERSTRASS) CUROB_RR_FIN(K_GRIEWANK) CUROB_RR_FIN(K_RASTRIGIN) CUROB_RR_FIN(K_F7)
    CUROB_RR_FIN(K_GRIEROSEN) CUROB_RR_FIN(K_ROSENBROCK) CUROB_RR_FIN(K_SCHWEFEL) CUROB_RR_FIN(K_KATSUURA)
    CUROB_RR_FIN(K_LUNACEK) CUROB_RR_FIN(K_ACKLEY) CUROB_RR_FIN(K_HAPPYCAT) CUROB_RR_FIN(K_HGBAT)
    CUROB_RR_FIN(K_F6)
#undef CUROB_RR_FIN
    default: return T(0);
  }
}

__device__ __forceinline__ float seg_param(const TiledSeg &sg) {
  if (sg.kind == K_SCHWEFEL) return static_cast<float>(1.0 / (10000.0 * static_cast<double>(sg.n)));
  if (sg.kind == K_KATSUURA) return static_cast<float>(sg.kparam);
  return 0.0f;
}

// Cuts 8 gathered y into the split path's bf16 terms (y - hi and the next residual are exact).
template <int NT>
__device__ __forceinline__ void cut8(const float (&y)[8], bf16x8 (&t)[NT]) {
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    const f32x2 v = {y[e], y[e + 1]};
    const bf16x2 h = __builtin_convertvector(v, bf16x2);
    const f32x2 r1 = v - __builtin_convertvector(h, f32x2);
    t[0][e] = h[0];
    t[0][e + 1] = h[1];
    if constexpr (NT == 3) {
      const bf16x2 m = __builtin_convertvector(r1, bf16x2);
      const bf16x2 l = __builtin_convertvector(r1 - __builtin_convertvector(m, f32x2), bf16x2);
      t[1][e] = m[0];
      t[1][e + 1] = m[1];
      t[2][e] = l[0];
      t[2][e + 1] = l[1];
    } else {
      const bf16x2 l = __builtin_convertvector(r1, bf16x2);
      t[1][e] = l[0];
      t[1][e + 1] = l[1];
    }
  }
}

// The split products of one (m-tile, column block) for one k step: A terms a[], B terms b[].
template <int NT>
__device__ __forceinline__ f32x4 products(const bf16x8 (&a)[NT], const bf16x8 (&b)[NT], f32x4 acc) {
  if constexpr (NT == 3) {
    // hi, mid, lo: the six products of order <= 2, smallest first
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[2], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], acc, 0, 0, 0);
  }
  return acc;
}

// Formula terms of one accumulator fragment (4 packed positions from pos) into the lane's
// running sums a; family K known at compile time.
template <int K>
__device__ __forceinline__ void terms(const f32x4 &acc, const f32x4 &cz, const f32x4 &cf, float prm, Acc<float> &a) {
  float v[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int e = 0; e < 4; ++e) phi<K, float>(v, a.p, acc[e] + cz[e], 0.0f, cf[e], prm);
#pragma unroll
  for (int k = 0; k < 3; ++k) acc_add<K, float>(a, k, v[k]);
}

// The same with the family read at run time (hybrid segments); pair families never get here.
__device__ __forceinline__ void terms_any(int kind, const f32x4 &acc, const f32x4 &cz, const f32x4 &cf, float prm,
                                          Acc<float> &a) {
  switch (kind) {
#define CUROB_RR_T(K) \
  case K: terms<K>(acc, cz, cf, prm, a); break;
    CUROB_RR_T(K_WSPHERE) CUROB_RR_T(K_POWERS) CUROB_RR_T(K_SHARPV) CUROB_RR_T(K_STEP) CUROB_RR_T(K_WEIERSTRASS)
    CUROB_RR_T(K_GRIEWANK) CUROB_RR_T(K_RASTRIGIN) CUROB_RR_T(K_SCHWEFEL) CUROB_RR_T(K_KATSUURA)
    CUROB_RR_T(K_LUNACEK) CUROB_RR_T(K_ACKLEY) CUROB_RR_T(K_HAPPYCAT) CUROB_RR_T(K_HGBAT)
#undef CUROB_RR_T
    default: break;
  }
}

// Merges the four lanes of a row (lane groups q = lane / 16) into lane group 0 and leaves the
// row's partial in the wave's LDS slot.
__device__ __forceinline__ void flush(Acc<float> &a, float *slot, int q) {
#pragma unroll
  for (int sh = 16; sh <= 32; sh <<= 1) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float so = __shfl_xor(a.s[k], sh, 64);
      const float co = __shfl_xor(a.c[k], sh, 64);
      acc_merge(a, k, so, co);
    }
    a.p *= __shfl_xor(a.p, sh, 64);
  }
  if (q == 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      slot[2 * k] = a.s[k];
      slot[2 * k + 1] = a.c[k];
    }
    slot[6] = a.p;
  }
  a.init();
}

// Pair terms of one pairwise segment for one row, from the packed z copy zr; lanes over the
// segment's positions.
template <int K>
__device__ __forceinline__ void pair_row(const TiledProb &tp, const TiledSeg &sg, const float *zr, float prm, int lane,
                                         Acc<float> &a) {
  const float *coefp = static_cast<const float *>(tp.coef);
  for (int p0 = sg.p0; p0 < sg.p1; p0 += 64) {
    const int pp = p0 + lane;
    const int pc = pp < sg.p1 ? pp : sg.p1 - 1;
    const int sp = tp.succ[pc];
    const int gi = tp.gidx[pc];
    const float z = zr[pc];
    const float zn = zr[sp >= 0 ? sp : pc];
    const float cf = coefp[pc];
    if (pp < sg.p1 && gi >= 0 && sp >= 0) {
      float v[3] = {0.0f, 0.0f, 0.0f};
      phi<K, float>(v, a.p, z, zn, cf, prm);
      a.add(0, v[0]);
    }
  }
}

__device__ __forceinline__ void pair_row_any(const TiledProb &tp, const TiledSeg &sg, const float *zr, float prm,
                                             int lane, Acc<float> &a) {
  switch (sg.kind) {
    case K_F7: pair_row<K_F7>(tp, sg, zr, prm, lane, a); break;
    case K_GRIEROSEN: pair_row<K_GRIEROSEN>(tp, sg, zr, prm, lane, a); break;
    case K_ROSENBROCK: pair_row<K_ROSENBROCK>(tp, sg, zr, prm, lane, a); break;
    case K_F6: pair_row<K_F6>(tp, sg, zr, prm, lane, a); break;
    default: break;
  }
}

// Buffer resource over rows [row0, n) of x: rows past n read as zeros.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rows_rsrc(const float *x, int row0, int n, int D) {
  const long long bytes = static_cast<long long>(n - row0) * D * 4LL;
  const int nb = bytes > 0x7ffffff0LL ? 0x7ffffff0 : (bytes > 0 ? static_cast<int>(bytes) : 0);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(x + static_cast<size_t>(row0) * D), (short)0, nb,
                                           0x00020000);
}

// One row (D floats at byte soff of the resource) into LDS at dst (16-byte aligned), with buffer
// loads that write LDS: 16 bytes per lane when wide (D a multiple of 4, rows 16-byte aligned in
// memory), 4 otherwise.  Lanes past the row's end are masked off, so nothing past column D - 1
// is written.
__device__ __forceinline__ void load_row(__amdgpu_buffer_rsrc_t rs, int D, float *dst, int soff, bool wide, int lane) {
  typedef __attribute__((address_space(3))) void *lds_ptr;
  if (wide) {
    for (int k0 = 0; k0 < D; k0 += 256)
      if (4 * lane < D - k0)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_ptr)(dst + k0), 16, (k0 + 4 * lane) * 4, soff, 0, 0);
  } else {
    for (int k0 = 0; k0 < D; k0 += 64)
      if (lane < D - k0)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_ptr)(dst + k0), 4, (k0 + lane) * 4, soff, 0, 0);
  }
}

constexpr int kWaitVmem = 0x3F70;  // s_waitcnt vmcnt(0), other counters free (gfx9 encoding)

// One problem (basic function or hybrid) on the rows staged in LDS: every rotation block, the
// formula terms and row sums, the pair terms.  Returns, in wave 0 lanes < 16 CB, the sum of the
// row's finalised segments (f without f_opt); other lanes return 0.  The problem's gather tables
// must be in s_goff / s_ohp.  Every barrier is reached by all waves.
// KIND >= 0: one formula family (basic functions); KIND < 0: family per segment at run time
// (hybrids, composition components).  NT: bf16 terms per operand (2: three products, 3: six).
// CB: 16-row column blocks (2; 1 when pair terms need the z copy s_z).
template <int NT, int KIND, int CB>
__device__ __forceinline__ float eval_tile(const TiledProb &tp, const float *s_rows, int S, const uint16_t *s_goff,
                                           const float *s_ohp, float *s_z, float *s_red, int lane, int wave) {
  constexpr int R = 16 * CB;
  constexpr bool PAIRS = CB == 1;
  const int r = lane & 15, q = lane >> 4;
  const int Dp = tp.Dp;
  const bf16x8 *qfrag = static_cast<const bf16x8 *>(tp.qfrag);
  const float *czp = static_cast<const float *>(tp.cz);
  const float *cfp = static_cast<const float *>(tp.coef);

  float F = 0.0f;
  Acc<float> a[CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) a[cb].init();
  int seg_open = -1;  // segment whose sums the waves are accumulating

  // merges the waves' sums of segment ps in wave order and finalises it (wave 0 keeps F)
  auto close_segment = [&](const TiledSeg &ps) {
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) flush(a[cb], s_red + (wave * R + 16 * cb + r) * kSlots, q);
    __syncthreads();
    if (wave == 0 && lane < R) {
      Acc<float> m;
      m.init();
      for (int w = 0; w < kWaves; ++w) {
        const float *src = s_red + (w * R + lane) * kSlots;
#pragma unroll
        for (int k = 0; k < 3; ++k) acc_merge(m, k, src[2 * k], src[2 * k + 1]);
        m.p *= src[6];
      }
      float sm[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) sm[k] = m.get_minus(k, ps.padc[k]);
      F += finalize_kind<float>(ps.kind, sm, m.p, ps.n);
    }
    __syncthreads();
  };

  for (int b = 0; b < tp.nblocks; ++b) {
    const int4 blk = tp.blocks[b];  // padded offset, padded size, first tile, k steps
    const int mts = blk.y >> 4, nst = blk.w;
    // the block's formula segment (one per block for hybrids, one overall for basics)
    int segi = 0;
    if constexpr (KIND < 0) {
      for (int si = 0; si < tp.nsegs; ++si)
        if (blk.x >= tp.segs[si].p0 && blk.x < tp.segs[si].p1) segi = si;
    }
    const TiledSeg &sg = tp.segs[segi];
    if (KIND < 0 && seg_open >= 0 && seg_open != segi && !tp.segs[seg_open].pairwise) close_segment(tp.segs[seg_open]);
    seg_open = segi;
    const int kind = KIND >= 0 ? KIND : sg.kind;
    const bool pairseg = KIND >= 0 ? KindTraits<(KIND >= 0 ? KIND : 0)>::pairwise : sg.pairwise != 0;
    const float prm = seg_param(sg);

    for (int mbase = wave; mbase < mts; mbase += kWaves * kMW) {
      // this pass: m-tiles mbase + kWaves j of the block (inactive ones recompute the first and
      // are discarded)
      int mt[kMW];
#pragma unroll
      for (int j = 0; j < kMW; ++j) mt[j] = mbase + kWaves * j < mts ? mbase + kWaves * j : mbase;
      const bf16x8 *qa[kMW];
#pragma unroll
      for (int j = 0; j < kMW; ++j) qa[j] = qfrag + static_cast<size_t>(blk.z + mt[j] * nst) * (NT * 64) + lane;
      f32x4 acc[kMW][CB];
#pragma unroll
      for (int j = 0; j < kMW; ++j)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[j][cb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      // rotation tiles two steps ahead: a0 holds even steps, a1 odd ones
      bf16x8 a0[kMW][NT], a1[kMW][NT];
#pragma unroll
      for (int j = 0; j < kMW; ++j)
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          a0[j][u] = qa[j][u * 64];
          a1[j][u] = qa[j][((nst > 1 ? 1 : 0) * NT + u) * 64];
        }
      auto step = [&](int c, bf16x8 (&au)[kMW][NT]) {
        // B: 8 packed positions per lane, gathered from the rows of each column block
        const int p0 = blk.x + 32 * c + 8 * q;
        const uint4 idx = *reinterpret_cast<const uint4 *>(s_goff + p0);
        const uint32_t iw[4] = {idx.x, idx.y, idx.z, idx.w};
        const f32x4 oa = *reinterpret_cast<const f32x4 *>(s_ohp + p0);
        const f32x4 ob = *reinterpret_cast<const f32x4 *>(s_ohp + p0 + 4);
        const float ov[8] = {oa[0], oa[1], oa[2], oa[3], ob[0], ob[1], ob[2], ob[3]};
        bf16x8 bt[CB][NT];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          const unsigned char *row = reinterpret_cast<const unsigned char *>(s_rows + (16 * cb + r) * S);
          float y[8];
#pragma unroll
          for (int e = 0; e < 8; e += 2) {
            y[e] = *reinterpret_cast<const float *>(row + (iw[e >> 1] & 0xFFFFu)) - ov[e];
            y[e + 1] = *reinterpret_cast<const float *>(row + (iw[e >> 1] >> 16)) - ov[e + 1];
          }
          cut8<NT>(y, bt[cb]);
        }
#pragma unroll
        for (int j = 0; j < kMW; ++j)
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) acc[j][cb] = products<NT>(au[j], bt[cb], acc[j][cb]);
        // this register set now takes step c + 2 (clamped: past the end it reloads the last)
        const int cn = c + 2 < nst ? c + 2 : nst - 1;
#pragma unroll
        for (int j = 0; j < kMW; ++j)
#pragma unroll
          for (int u = 0; u < NT; ++u) au[j][u] = qa[j][(static_cast<size_t>(cn) * NT + u) * 64];
      };
      for (int c = 0; c < nst; c += 2) {
        step(c, a0);
        if (c + 1 < nst) step(c + 1, a1);
      }
      // epilogue: z = acc + c' per position; terms into the wave's row sums, or z into the
      // packed copy for pair terms
#pragma unroll
      for (int j = 0; j < kMW; ++j) {
        if (mbase + kWaves * j >= mts) continue;
        const int pm = blk.x + 16 * mt[j] + 4 * q;  // 4 consecutive packed positions
        const f32x4 cz4 = *reinterpret_cast<const f32x4 *>(czp + pm);
        if (pairseg) {
          if constexpr (PAIRS) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) *reinterpret_cast<f32x4 *>(s_z + (16 * cb + r) * Dp + pm) = acc[j][cb] + cz4;
          }
        } else {
          const f32x4 cf4 = *reinterpret_cast<const f32x4 *>(cfp + pm);
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
            if constexpr (KIND >= 0) terms<(KIND >= 0 ? KIND : 0)>(acc[j][cb], cz4, cf4, prm, a[cb]);
            else terms_any(kind, acc[j][cb], cz4, cf4, prm, a[cb]);
          }
        }
      }
    }
  }
  // the last open segment (every segment of a basic function)
  {
    const TiledSeg &ps = tp.segs[seg_open >= 0 ? seg_open : 0];
    if (!ps.pairwise) close_segment(ps);
    else __syncthreads();
  }
  if constexpr (PAIRS) {
    // pair terms from the z copy: each wave takes rows, lanes the positions of each pairwise
    // segment; the row's pair value goes to slot 0 of its partials (no other use now)
    for (int rr = wave; rr < R; rr += kWaves) {
      float fr = 0.0f;
      for (int si = 0; si < tp.nsegs; ++si) {
        const TiledSeg &ps = tp.segs[si];
        if (!ps.pairwise) continue;
        Acc<float> m;
        m.init();
        pair_row_any(tp, ps, s_z + rr * Dp, seg_param(ps), lane, m);
#pragma unroll
        for (int sh = 1; sh < 64; sh <<= 1) {
          const float so = __shfl_xor(m.s[0], sh, 64);
          const float co = __shfl_xor(m.c[0], sh, 64);
          acc_merge(m, 0, so, co);
        }
        float sm[3] = {m.get_minus(0, ps.padc[0]), 0.0f, 0.0f};
        fr += finalize_kind<float>(ps.kind, sm, 1.0f, ps.n);
      }
      if (lane == 0) s_red[rr * kSlots] = fr;
    }
    __syncthreads();
    if (wave == 0 && lane < R) F += s_red[lane * kSlots];
    __syncthreads();
  }
  return F;
}

// Loads the gather tables of problem tp into LDS (all threads).
__device__ __forceinline__ void load_tables(const TiledProb &tp, uint16_t *s_goff, float *s_ohp) {
  for (int i = threadIdx.x; i < tp.Dp; i += kThreads) {
    s_goff[i] = tp.goff[i];
    s_ohp[i] = tp.ohp[i];
  }
}

// Stages rows [row0, row0 + R) of x (R = 16 CB; past n: zeros) at stride S, then barrier.
template <int CB>
__device__ __forceinline__ void stage_rows(const float *x, int row0, int n, int D, int S, float *s_rows, bool wide,
                                           int lane, int wave) {
  constexpr int R = 16 * CB;
  const __amdgpu_buffer_rsrc_t rs = rows_rsrc(x, row0, n, D);
  for (int rr = wave; rr < R; rr += kWaves) load_row(rs, D, s_rows + rr * S, rr * 4 * D, wide, lane);
  __builtin_amdgcn_s_waitcnt(kWaitVmem);
  __syncthreads();
}

// Basic function or hybrid: persistent grid over tiles of 16 CB rows.
template <int P, int KIND, int CB>
__global__ __launch_bounds__(kThreads) void k_rowres(TiledProb tp, const float *__restrict__ x, int n,
                                                     float *__restrict__ out, int wide) {
  constexpr int R = 16 * CB;
  extern __shared__ __align__(16) unsigned char smem[];
  const int D = tp.D, S = tp.S;
  const Carve L = carve(tp.Dp, S, CB, CB == 1);
  uint16_t *s_goff = reinterpret_cast<uint16_t *>(smem + L.goff);
  float *s_ohp = reinterpret_cast<float *>(smem + L.ohp);
  float *s_rows = reinterpret_cast<float *>(smem + L.rows);
  float *s_z = reinterpret_cast<float *>(smem + L.zc);
  float *s_red = reinterpret_cast<float *>(smem + L.red);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  load_tables(tp, s_goff, s_ohp);
  // the zero slot (column D) of every row: padded positions gather it; loads never write it
  if (threadIdx.x < R) s_rows[threadIdx.x * S + D] = 0.0f;
  const int ntiles = (n + R - 1) / R;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int row0 = tile * R;
    __syncthreads();  // the previous tile's readers of the rows are done
    stage_rows<CB>(x, row0, n, D, S, s_rows, wide != 0, lane, wave);
    const float F = eval_tile<split_terms(P), KIND, CB>(tp, s_rows, S, s_goff, s_ohp, s_z, s_red, lane, wave);
    if (wave == 0 && lane < R && row0 + lane < n) out[row0 + lane] = F + static_cast<float>(tp.bias);
  }
}

// One component of a fused composition: its tiled tables (device copy) and arithmetic.
struct CompDesc {
  TiledProb tp;
  int six;        // split mode: six products
  int unrotated;  // z = s (x - o_hi) + c' per variable, no rotation (no pair terms)
};

// Unrotated component on the staged rows: each wave takes rows, lanes the variables; returns the
// component value in wave 0 lanes < R (through s_red).
template <int CB>
__device__ __forceinline__ float eval_unrotated(const TiledProb &tp, const float *s_rows, int S, float *s_red, int lane,
                                                int wave) {
  constexpr int R = 16 * CB;
  const float s = static_cast<float>(tp.scale0);
  const float *oh = static_cast<const float *>(tp.oh);
  const float *czp = static_cast<const float *>(tp.cz);
  const float *cfp = static_cast<const float *>(tp.coef);
  const TiledSeg &sg = tp.segs[0];
  const float prm = seg_param(sg);
  for (int rr = wave; rr < R; rr += kWaves) {
    Acc<float> m;
    m.init();
    for (int j0 = 0; j0 < tp.D; j0 += 64) {
      const int j = j0 + lane;
      const int jc = j < tp.D ? j : tp.D - 1;
      const float z = s * (s_rows[rr * S + jc] - oh[jc]) + czp[jc];
      if (j < tp.D) {
        float v[3] = {0.0f, 0.0f, 0.0f};
        switch (sg.kind) {
#define CUROB_RR_U(K) \
  case K: phi<K, float>(v, m.p, z, 0.0f, cfp[jc], prm); break;
          CUROB_RR_U(K_WSPHERE) CUROB_RR_U(K_POWERS) CUROB_RR_U(K_SHARPV) CUROB_RR_U(K_STEP)
          CUROB_RR_U(K_WEIERSTRASS) CUROB_RR_U(K_GRIEWANK) CUROB_RR_U(K_RASTRIGIN) CUROB_RR_U(K_SCHWEFEL)
          CUROB_RR_U(K_KATSUURA) CUROB_RR_U(K_LUNACEK) CUROB_RR_U(K_ACKLEY) CUROB_RR_U(K_HAPPYCAT)
          CUROB_RR_U(K_HGBAT)
#undef CUROB_RR_U
          default: break;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) m.add(k, v[k]);
      }
    }
#pragma unroll
    for (int sh = 1; sh < 64; sh <<= 1) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float so = __shfl_xor(m.s[k], sh, 64);
        const float co = __shfl_xor(m.c[k], sh, 64);
        acc_merge(m, k, so, co);
      }
      m.p *= __shfl_xor(m.p, sh, 64);
    }
    if (lane == 0) {
      float sm[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) sm[k] = m.get(k);
      s_red[rr * kSlots] = finalize_kind<float>(sg.kind, sm, m.p, sg.n);
    }
  }
  __syncthreads();
  const float F = (wave == 0 && lane < R) ? s_red[lane * kSlots] : 0.0f;
  __syncthreads();
  return F;
}

// LDS carve of the fused composition: the row carve for the largest component tables, then the
// component values (FP32) and squared distances (FP64) per (component, row).
struct CompCarve {
  Carve base;
  int g, d2, total;
};
__host__ __device__ inline CompCarve comp_carve(int Dpmax, int S, int CB) {
  CompCarve c;
  c.base = carve(Dpmax, S, CB, CB == 1);
  const int R = 16 * CB;
  c.g = c.base.total;
  c.d2 = c.g + round16(8 * R * 4);
  c.total = c.d2 + 8 * R * 8;
  return c;
}

// Composition (Sec. 6, Eqs. (composition) and (weight)) with every component on the same staged
// rows: X is read from HBM once.  Per tile: each component's value G_i (its gather tables loaded
// into LDS in turn, f_opt excluded), then d_i^2 = |x - o^i|^2 in FP64 from the staged FP32 rows,
// log-domain weights in FP64 (one-hot where some d_i = 0), F = sum omega_i (lambda_i G_i + bias_i)
// + f_opt.
template <int CB>
__global__ __launch_bounds__(kThreads) void k_rowres_comp(const CompDesc *__restrict__ comps, int nc, int Dpmax,
                                                          int S, const float *__restrict__ x, int n, int D,
                                                          const double *__restrict__ o64,
                                                          const double *__restrict__ sigma,
                                                          const double *__restrict__ lambda,
                                                          const double *__restrict__ bias, double fopt,
                                                          float *__restrict__ out, int wide) {
  constexpr int R = 16 * CB;
  extern __shared__ __align__(16) unsigned char smem[];
  const CompCarve L = comp_carve(Dpmax, S, CB);
  uint16_t *s_goff = reinterpret_cast<uint16_t *>(smem + L.base.goff);
  float *s_ohp = reinterpret_cast<float *>(smem + L.base.ohp);
  float *s_rows = reinterpret_cast<float *>(smem + L.base.rows);
  float *s_z = reinterpret_cast<float *>(smem + L.base.zc);
  float *s_red = reinterpret_cast<float *>(smem + L.base.red);
  float *s_g = reinterpret_cast<float *>(smem + L.g);
  double *s_d2 = reinterpret_cast<double *>(smem + L.d2);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (threadIdx.x < R) s_rows[threadIdx.x * S + D] = 0.0f;
  const int ntiles = (n + R - 1) / R;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int row0 = tile * R;
    __syncthreads();
    stage_rows<CB>(x, row0, n, D, S, s_rows, wide != 0, lane, wave);
    for (int i = 0; i < nc; ++i) {
      const CompDesc &cd = comps[i];
      float G;
      if (cd.unrotated) {
        G = eval_unrotated<CB>(cd.tp, s_rows, S, s_red, lane, wave);
      } else {
        __syncthreads();  // the previous component's readers of the tables are done
        load_tables(cd.tp, s_goff, s_ohp);
        __syncthreads();
        if (cd.six) G = eval_tile<3, -1, CB>(cd.tp, s_rows, S, s_goff, s_ohp, s_z, s_red, lane, wave);
        else G = eval_tile<2, -1, CB>(cd.tp, s_rows, S, s_goff, s_ohp, s_z, s_red, lane, wave);
      }
      if (wave == 0 && lane < R) s_g[i * R + lane] = G;
    }
    // squared distances to every optimum in FP64 (the FP32 rows widen exactly): each wave takes
    // rows, lanes the variables
    for (int rr = wave; rr < R; rr += kWaves) {
      for (int i = 0; i < nc; ++i) {
        double acc = 0.0;
        for (int j = lane; j < D; j += 64) {
          const double d = static_cast<double>(s_rows[rr * S + j]) - o64[static_cast<size_t>(i) * D + j];
          acc += d * d;
        }
#pragma unroll
        for (int sh = 1; sh < 64; sh <<= 1) acc += __shfl_xor(acc, sh, 64);
        if (lane == 0) s_d2[i * R + rr] = acc;
      }
    }
    __syncthreads();
    if (wave == 0 && lane < R && row0 + lane < n) {
      int nzero = 0;
      double amax = -1.0e308;
      for (int i = 0; i < nc; ++i) {
        const double d2 = s_d2[i * R + lane];
        if (d2 == 0.0) ++nzero;
        else amax = fmax(amax, -0.5 * log(d2) - d2 / (2.0 * D * sigma[i] * sigma[i]));
      }
      double wsum = 0.0, g = 0.0;
      for (int i = 0; i < nc; ++i) {
        const double d2 = s_d2[i * R + lane];
        const double w = nzero ? (d2 == 0.0 ? 1.0 : 0.0)
                               : exp(-0.5 * log(d2) - d2 / (2.0 * D * sigma[i] * sigma[i]) - amax);
        wsum += w;
        g += w * (lambda[i] * static_cast<double>(s_g[i * R + lane]) + bias[i]);
      }
      out[row0 + lane] = static_cast<float>(g / wsum + fopt);
    }
  }
}

}  // namespace rowres

}  // namespace curob
