// eval_rowres.h -- fused evaluation for dimensions above the resident kernel's range on the
// split paths (basic functions and hybrids, Sec. 5; the components of a composition, Sec. 6),
// with the population rows resident in LDS.
//
// A workgroup of eight waves holds 32 population rows in LDS (x as read) and computes every
// output of the packed block-diagonal rotation for them:
//   - for each rotation block, each wave takes up to three m-tiles (16 outputs) of the block per
//     pass (four when a block has 25..32 m-tiles, so that it takes one pass) and all waves walk
//     the block's k steps together.  The B operand of a k step (y = x - o_hi at
//     32 packed positions for the 32 rows, cut into bf16 terms) is produced once per workgroup,
//     one pair of positions of one row per thread, into a two-slot LDS ring in MFMA operand
//     order, one barrier per step; every wave then reads it with one 16-byte LDS read per
//     (column block, term).  The rotation tiles (A operand) stream from L2 through buffer loads
//     issued several steps ahead of their products (four for three products, three for six,
//     one less with four m-tiles per wave);
//   - z = acc + c' then the formula's per-element terms go into the wave's compensated row
//     sums.  Formulas with pair terms instead write z back into the LDS rows, at the slot of
//     the position's own variable (the block's variables are read by no later step), and the
//     pair terms are summed from there once every block is done;
//   - row sums of all waves meet in LDS, in wave order, and wave 0 finalises each formula
//     segment of its rows.
// The rows reach LDS through buffer loads that write LDS directly; for problems without pair
// terms the next tile's rows are requested as soon as the current tile's last rotation step has
// read its rows.  X is read from HBM once, nothing goes through scratch memory, and the result
// row is written directly.  Persistent grid: each workgroup walks row tiles with a stride of the
// grid.
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
constexpr int kMW = 3;      // m-tiles of one block per wave pass (one B chunk feeds them all)
constexpr int kMWWide = 4;  // the same for problems with a block of 25..32 m-tiles (hybrid groups)
constexpr int kSlots = 8;   // per (wave, row) partial: s0 c0 s1 c1 s2 c2 product pad
constexpr int kCB = 2;      // 16-row column blocks per tile
constexpr int kRows = 16 * kCB;
// m-tiles one pass covers; a block with pair terms must fit one pass (its z overwrites rows
// that a second pass would read again)
constexpr int kPassMTiles = kWaves * kMW;

// Bytes of one ring slot: kCB column blocks x NT terms x 64 lanes x 16 bytes.
__host__ __device__ constexpr int ring_slot_bytes(int NT) { return kCB * NT * 64 * 16; }

// Rows this wide fit the LDS carve next to the tables, the ring and the partials.
constexpr int kMaxD = 1088;

// LDS carve: packed-position tables, the rows, the B ring, the per-wave partials.
struct Carve {
  int goff, ohp, rows, ring, red, total;
};
__host__ __device__ inline Carve carve(int Dp, int S, int NT) {
  Carve c;
  c.goff = 0;
  c.ohp = round16(Dp * 2);
  c.rows = c.ohp + round16(Dp * 4);
  c.ring = c.rows + round16(kRows * S * 4);
  c.red = c.ring + 2 * ring_slot_bytes(NT);
  c.total = c.red + kWaves * kRows * kSlots * 4;
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

// Product st of products<NT> alone (st fixed at compile time after unrolling).
template <int NT>
__device__ __forceinline__ f32x4 product_stage(int st, const bf16x8 (&a)[NT], const bf16x8 (&b)[NT], f32x4 acc) {
  if constexpr (NT == 3) {
    constexpr int ia[6] = {2, 1, 0, 1, 0, 0}, ib[6] = {0, 1, 2, 0, 1, 0};
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ia[st]], b[ib[st]], acc, 0, 0, 0);
  } else {
    constexpr int ia[3] = {1, 0, 0}, ib[3] = {0, 1, 0};
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ia[st]], b[ib[st]], acc, 0, 0, 0);
  }
}

// Cuts the pair y of one thread's share of a B step into NT bf16 terms (y - hi and the next
// residual are exact in FP32) and writes them at dst, the pair's place in a ring slot: term u of
// lane slot l of column block cb sits at byte ((cb NT + u) 64 + l) 16 of the slot, the 16-byte
// B fragment of that MFMA lane (the 32 positions x 32 rows of a step: 512 threads, one pair each).
template <int NT>
__device__ __forceinline__ void cut_pair(unsigned char *dst, f32x2 y) {
  const bf16x2 h = __builtin_convertvector(y, bf16x2);
  const f32x2 r1 = y - __builtin_convertvector(h, f32x2);
  *reinterpret_cast<uint32_t *>(dst) = __builtin_bit_cast(uint32_t, h);
  if constexpr (NT == 3) {
    const bf16x2 m = __builtin_convertvector(r1, bf16x2);
    const bf16x2 lo = __builtin_convertvector(r1 - __builtin_convertvector(m, f32x2), bf16x2);
    *reinterpret_cast<uint32_t *>(dst + 64 * 16) = __builtin_bit_cast(uint32_t, m);
    *reinterpret_cast<uint32_t *>(dst + 2 * 64 * 16) = __builtin_bit_cast(uint32_t, lo);
  } else {
    const bf16x2 lo = __builtin_convertvector(r1, bf16x2);
    *reinterpret_cast<uint32_t *>(dst + 64 * 16) = __builtin_bit_cast(uint32_t, lo);
  }
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

// Pair terms of one pairwise segment for the wave's rows (kRows / kWaves of them, rows wave +
// kWaves i), from z written back over the rows' x at the slot of each position's variable; lanes
// take the segment's positions.  A position's successor and variable are read once for all the
// wave's rows, and those of the next 64 positions are requested before the current ones' terms.
constexpr int kPairRows = kRows / kWaves;
static_assert(kPairRows * kWaves == kRows, "pair terms: whole rows per wave");
template <int K>
__device__ __forceinline__ void pair_rows(const TiledProb &tp, const TiledSeg &sg, const float *s_rows, int S,
                                          const uint16_t *s_goff, float prm, int lane, int wave,
                                          Acc<float> (&m)[kPairRows]) {
  auto clampp = [&](int pp) { return pp < sg.p1 ? pp : sg.p1 - 1; };
  int sp = tp.succ[clampp(sg.p0 + lane)];
  int gi = tp.gidx[clampp(sg.p0 + lane)];
  for (int p0 = sg.p0; p0 < sg.p1; p0 += 64) {
    const int pp = p0 + lane;
    const int pc = clampp(pp);
    const bool live = pp < sg.p1 && gi >= 0 && sp >= 0;
    const uint32_t go = s_goff[pc];
    const uint32_t gn = s_goff[sp >= 0 ? sp : pc];
    const int pn = clampp(p0 + 64 + lane);
    const int sp2 = tp.succ[pn];
    const int gi2 = tp.gidx[pn];
#pragma unroll
    for (int i = 0; i < kPairRows; ++i) {
      const unsigned char *zr = reinterpret_cast<const unsigned char *>(s_rows + (wave + kWaves * i) * S);
      const float z = *reinterpret_cast<const float *>(zr + go);
      const float zn = *reinterpret_cast<const float *>(zr + gn);
      if (live) {
        float v[3] = {0.0f, 0.0f, 0.0f};
        phi<K, float>(v, m[i].p, z, zn, 0.0f, prm);
        m[i].add(0, v[0]);
      }
    }
    sp = sp2;
    gi = gi2;
  }
}

__device__ __forceinline__ void pair_rows_any(const TiledProb &tp, const TiledSeg &sg, const float *s_rows, int S,
                                              const uint16_t *s_goff, float prm, int lane, int wave,
                                              Acc<float> (&m)[kPairRows]) {
  switch (sg.kind) {
    case K_F7: pair_rows<K_F7>(tp, sg, s_rows, S, s_goff, prm, lane, wave, m); break;
    case K_GRIEROSEN: pair_rows<K_GRIEROSEN>(tp, sg, s_rows, S, s_goff, prm, lane, wave, m); break;
    case K_ROSENBROCK: pair_rows<K_ROSENBROCK>(tp, sg, s_rows, S, s_goff, prm, lane, wave, m); break;
    case K_F6: pair_rows<K_F6>(tp, sg, s_rows, S, s_goff, prm, lane, wave, m); break;
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
// The loads are non-temporal (cache policy nt): the population streams through once and should
// not evict the rotation tiles, which every tile re-reads from L2.
constexpr int kCachePolicyNT = 2;
__device__ __forceinline__ void load_row(__amdgpu_buffer_rsrc_t rs, int D, float *dst, int soff, bool wide, int lane) {
  typedef __attribute__((address_space(3))) void *lds_ptr;
  if (wide) {
    for (int k0 = 0; k0 < D; k0 += 256)
      if (4 * lane < D - k0)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_ptr)(dst + k0), 16, (k0 + 4 * lane) * 4, soff, 0,
                                                 kCachePolicyNT);
  } else {
    for (int k0 = 0; k0 < D; k0 += 64)
      if (lane < D - k0)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_ptr)(dst + k0), 4, (k0 + lane) * 4, soff, 0, kCachePolicyNT);
  }
}

constexpr int kWaitVmem = 0x3F70;  // s_waitcnt vmcnt(0), other counters free (gfx9 encoding)

// Issues the loads that bring rows [row0, row0 + 32) of x (past n: zeros) into LDS at stride S.
__device__ __forceinline__ void issue_rows(const float *x, int row0, int n, int D, int S, float *s_rows, bool wide,
                                           int lane, int wave) {
  const __amdgpu_buffer_rsrc_t rs = rows_rsrc(x, row0, n, D);
  for (int rr = wave; rr < kRows; rr += kWaves) load_row(rs, D, s_rows + rr * S, rr * 4 * D, wide, lane);
}

// Waits for the rows issue_rows requested, rewrites the zero slot (column D) of every row, which
// padded positions gather, then barrier.
__device__ __forceinline__ void finish_rows(int D, int S, float *s_rows) {
  if (threadIdx.x < kRows) s_rows[threadIdx.x * S + D] = 0.0f;
  __builtin_amdgcn_s_waitcnt(kWaitVmem);
  __syncthreads();
}

__device__ __forceinline__ void stage_rows(const float *x, int row0, int n, int D, int S, float *s_rows, bool wide,
                                           int lane, int wave) {
  issue_rows(x, row0, n, D, S, s_rows, wide, lane, wave);
  finish_rows(D, S, s_rows);
}

// The rows of the workgroup's next tile, requested as soon as the last rotation step of the
// current tile has read its rows (row0 < 0: none, or the problem has pair terms, whose z stays
// in the rows until the end of the tile).
struct NextRows {
  const float *x;
  int row0, n, D;
  bool wide;
};

// One problem (basic function or hybrid) on the rows staged in LDS: every rotation block, the
// formula terms and row sums, the pair terms.  Returns, in wave 0 lanes < 32, the sum of the
// row's finalised segments (f without f_opt); other lanes return 0.  The problem's gather tables
// must be in s_goff / s_ohp.  Formulas with pair terms overwrite the x of their own variables
// with z.  Every barrier is reached by all threads.
// KIND >= 0: one formula family (basic functions); KIND < 0: family per segment at run time
// (hybrids, composition components).  NT: bf16 terms per operand (2: three products, 3: six).
// AHEAD: steps the rotation tiles are requested ahead of their products (registers permitting).
// LEAN (the fused composition kernel, short of registers): the epilogue reads its tables itself.
// MW: m-tiles per wave and pass.  Every step costs its B production and barrier whatever the
// m-tiles it feeds, so a block of 25..32 m-tiles (a wide hybrid group) takes one pass of four
// per wave instead of two passes of three (the fourth slot is idle in smaller blocks).
template <int NT, int KIND, int AHEAD, bool LEAN = false, int MW = kMW>
__device__ __forceinline__ float eval_tile(const TiledProb &tp, float *s_rows, int S, const uint16_t *s_goff,
                                           const float *s_ohp, unsigned char *s_ring, float *s_red, int lane,
                                           int wave, const NextRows &nx) {
  const int r = lane & 15, q = lane >> 4;
  const float *czp = static_cast<const float *>(tp.cz);
  const float *cfp = static_cast<const float *>(tp.coef);
  constexpr int kSlot = ring_slot_bytes(NT);
  const __amdgpu_buffer_rsrc_t qrs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(tp.qfrag), (short)0, 0x7ffffff0, 0x00020000);
  // this thread's share of each B step: column block t / 256, lane slot l = (t / 4) % 64 (row
  // l % 16, positions 8 (l / 16) ..), position pair e = 2 (t % 4), e + 1
  const int pt = static_cast<int>(threadIdx.x);
  const int pcb = pt >> 8, pl = (pt >> 2) & 63, pe = (pt & 3) * 2;
  const int pair_pos = 8 * (pl >> 4) + pe;
  const int pair_slot = ((pcb * NT) * 64 + pl) * 16 + pe * 2;
  const unsigned char *prow = reinterpret_cast<const unsigned char *>(s_rows + (16 * pcb + (pl & 15)) * S);

  float F = 0.0f;
  Acc<float> a[kCB];
#pragma unroll
  for (int cb = 0; cb < kCB; ++cb) a[cb].init();
  int seg_open = -1;  // segment whose sums the waves are accumulating
  bool any_pairs = false;

  // merges the waves' sums of segment ps in wave order and finalises it (wave 0 keeps F)
  auto close_segment = [&](const TiledSeg &ps) {
#pragma unroll
    for (int cb = 0; cb < kCB; ++cb) flush(a[cb], s_red + (wave * kRows + 16 * cb + r) * kSlots, q);
    __syncthreads();
    if (wave == 0 && lane < kRows) {
      Acc<float> m;
      m.init();
      for (int w = 0; w < kWaves; ++w) {
        const float *src = s_red + (w * kRows + lane) * kSlots;
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
    any_pairs = any_pairs || pairseg;
    const float prm = seg_param(sg);
    const int npass = (mts + (kWaves * MW) - 1) / (kWaves * MW);

    for (int pass = 0; pass < npass; ++pass) {
      // this pass: m-tiles mbase + kWaves j of the block.  A slot past the block's m-tiles
      // repeats the last m-tile and is discarded (no branch splits the step: waves 4 apart
      // share a SIMD, and the fullest SIMD sets the pace anyway)
      const int mbase = pass * (kWaves * MW) + wave;
      int mt[MW];
      bool act[MW];
#pragma unroll
      for (int j = 0; j < MW; ++j) {
        act[j] = mbase + kWaves * j < mts;
        mt[j] = act[j] ? mbase + kWaves * j : mts - 1;
      }
      // the epilogue's per-position tables, read now: no global load follows the next tile's
      // row requests, whose completion a later load would otherwise wait for
      f32x4 cz4[MW], cf4[MW];
      auto read_epi = [&]() {
#pragma unroll
        for (int j = 0; j < MW; ++j) {
          const int pm = blk.x + 16 * mt[j] + 4 * q;  // 4 consecutive packed positions
          cz4[j] = *reinterpret_cast<const f32x4 *>(czp + pm);
          cf4[j] = *reinterpret_cast<const f32x4 *>(cfp + pm);
        }
      };
      if constexpr (!LEAN) read_epi();
      // rotation tiles through buffer loads: per-lane offset fixed, tile offset scalar
      auto load_a = [&](bf16x8 (&au)[MW][NT], int c) {
#pragma unroll
        for (int j = 0; j < MW; ++j) {
          const int toff = (blk.z + mt[j] * nst + c) * (NT * 1024);
#pragma unroll
          for (int u = 0; u < NT; ++u)
            au[j][u] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(qrs, lane * 16 + u * 1024, toff, 0));
        }
      };
      f32x4 acc[MW][kCB];
#pragma unroll
      for (int j = 0; j < MW; ++j)
#pragma unroll
        for (int cb = 0; cb < kCB; ++cb) acc[j][cb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      // rotation tiles kAhead steps ahead: register set k holds the steps c with c % kAhead == k
      // (the loads of a step are in flight while the kAhead - 1 steps before it compute)
      constexpr int kAhead = AHEAD;
      bf16x8 ar[kAhead][MW][NT];
#pragma unroll
      for (int k = 0; k < kAhead; ++k) load_a(ar[k], k < nst ? k : nst - 1);
      // B operand pipeline (one barrier per step): step c consumes ring slot c & 1, gathers the
      // x of step c + 1 with offsets read one step earlier, reads the offsets of step c + 2, and
      // writes step c + 1 into the other slot (read last at step c - 1, before the previous
      // barrier).  Steps past the block repeat its last step into a slot nobody reads.
      auto pos = [&](int c) { return blk.x + 32 * (c < nst ? c : nst - 1) + pair_pos; };
      uint32_t go = *reinterpret_cast<const uint32_t *>(s_goff + pos(0));
      f32x2 oo = *reinterpret_cast<const f32x2 *>(s_ohp + pos(0));
      {
        const f32x2 y = f32x2{*reinterpret_cast<const float *>(prow + (go & 0xFFFFu)),
                              *reinterpret_cast<const float *>(prow + (go >> 16))} - oo;
        cut_pair<NT>(s_ring + pair_slot, y);
      }
      go = *reinterpret_cast<const uint32_t *>(s_goff + pos(1));
      oo = *reinterpret_cast<const f32x2 *>(s_ohp + pos(1));
      __syncthreads();
      auto step = [&](int c, bf16x8 (&au)[MW][NT]) {
        const unsigned char *slot = s_ring + (c & 1) * kSlot;
        bf16x8 bt[kCB][NT];
#pragma unroll
        for (int cb = 0; cb < kCB; ++cb)
#pragma unroll
          for (int u = 0; u < NT; ++u) bt[cb][u] = *reinterpret_cast<const bf16x8 *>(slot + ((cb * NT + u) * 64 + lane) * 16);
        const f32x2 xv = f32x2{*reinterpret_cast<const float *>(prow + (go & 0xFFFFu)),
                               *reinterpret_cast<const float *>(prow + (go >> 16))};
        const uint32_t go2 = *reinterpret_cast<const uint32_t *>(s_goff + pos(c + 2));
        const f32x2 oo2 = *reinterpret_cast<const f32x2 *>(s_ohp + pos(c + 2));
        __builtin_amdgcn_sched_barrier(0);
        // the product stages outermost: MW * kCB independent accumulators between two
        // products into the same one
#pragma unroll
        for (int st = 0; st < (NT == 3 ? 6 : 3); ++st)
#pragma unroll
          for (int j = 0; j < MW; ++j)
#pragma unroll
            for (int cb = 0; cb < kCB; ++cb) acc[j][cb] = product_stage<NT>(st, au[j], bt[cb], acc[j][cb]);
        // this register set now takes step c + kAhead (clamped: past the end it reloads the last)
        load_a(au, c + kAhead < nst ? c + kAhead : nst - 1);
        __builtin_amdgcn_sched_barrier(0);
        cut_pair<NT>(s_ring + ((c + 1) & 1) * kSlot + pair_slot, xv - oo);
        go = go2;
        oo = oo2;
        __syncthreads();
      };
      // whole rounds of kAhead steps without a branch (so the wait for a step's tiles counts
      // only the loads issued before them), then the remaining steps
      int c = 0;
      for (; c + kAhead <= nst; c += kAhead) {
#pragma unroll
        for (int k = 0; k < kAhead; ++k) step(c + k, ar[k]);
      }
#pragma unroll
      for (int k = 0; k < kAhead - 1; ++k)
        if (c + k < nst) step(c + k, ar[k]);
      // every read of the rows is done (the last step ended with a barrier)
      if (nx.row0 >= 0 && b == tp.nblocks - 1 && pass == npass - 1)
        issue_rows(nx.x, nx.row0, nx.n, nx.D, S, s_rows, nx.wide, lane, wave);
      // epilogue: z = acc + c' per position; terms into the wave's row sums, or z over the x of
      // the position's variable for pair terms (padding: z = 0 into the zero slot, unchanged)
      if constexpr (LEAN) read_epi();
#pragma unroll
      for (int j = 0; j < MW; ++j) {
        if (!act[j]) continue;
        const int pm = blk.x + 16 * (mbase + kWaves * j) + 4 * q;  // 4 consecutive packed positions
        if (pairseg) {
          const uint2 g2 = *reinterpret_cast<const uint2 *>(s_goff + pm);
          const uint32_t go[4] = {g2.x & 0xFFFFu, g2.x >> 16, g2.y & 0xFFFFu, g2.y >> 16};
#pragma unroll
          for (int cb = 0; cb < kCB; ++cb) {
            unsigned char *row = reinterpret_cast<unsigned char *>(s_rows + (16 * cb + r) * S);
            const f32x4 z = acc[j][cb] + cz4[j];
#pragma unroll
            for (int e = 0; e < 4; ++e) *reinterpret_cast<float *>(row + go[e]) = z[e];
          }
        } else {
#pragma unroll
          for (int cb = 0; cb < kCB; ++cb) {
            if constexpr (KIND >= 0) terms<(KIND >= 0 ? KIND : 0)>(acc[j][cb], cz4[j], cf4[j], prm, a[cb]);
            else terms_any(kind, acc[j][cb], cz4[j], cf4[j], prm, a[cb]);
          }
        }
      }
    }
  }
  // the last open segment (every segment of a basic function); the barrier also orders the z
  // written back above before the pair terms read it
  {
    const TiledSeg &ps = tp.segs[seg_open >= 0 ? seg_open : 0];
    if (!ps.pairwise) close_segment(ps);
    else __syncthreads();
  }
  if (any_pairs) {
    // pair terms: each wave takes rows, lanes the positions of each pairwise segment; the row's
    // pair value goes to slot 0 of its partials (no other use now)
    float fr[kPairRows];
#pragma unroll
    for (int i = 0; i < kPairRows; ++i) fr[i] = 0.0f;
    for (int si = 0; si < tp.nsegs; ++si) {
      const TiledSeg &ps = tp.segs[si];
      if (!ps.pairwise) continue;
      Acc<float> m[kPairRows];
#pragma unroll
      for (int i = 0; i < kPairRows; ++i) m[i].init();
      pair_rows_any(tp, ps, s_rows, S, s_goff, seg_param(ps), lane, wave, m);
#pragma unroll
      for (int i = 0; i < kPairRows; ++i) {
#pragma unroll
        for (int sh = 1; sh < 64; sh <<= 1) {
          const float so = __shfl_xor(m[i].s[0], sh, 64);
          const float co = __shfl_xor(m[i].c[0], sh, 64);
          acc_merge(m[i], 0, so, co);
        }
        float sm[3] = {m[i].get_minus(0, ps.padc[0]), 0.0f, 0.0f};
        fr[i] += finalize_kind<float>(ps.kind, sm, 1.0f, ps.n);
      }
    }
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < kPairRows; ++i) s_red[(wave + kWaves * i) * kSlots] = fr[i];
    }
    __syncthreads();
    if (wave == 0 && lane < kRows) F += s_red[lane * kSlots];
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

// Basic function or hybrid: persistent grid over tiles of 32 rows.  MW: m-tiles per wave and
// pass (kMWWide for a block of 25..32 m-tiles, with the rotation tiles one step less ahead to
// stay within the registers).
template <int NT, int KIND, int MW = kMW>
__global__ __launch_bounds__(kThreads) void k_rowres(TiledProb tp, const float *__restrict__ x, int n,
                                                     float *__restrict__ out, int wide) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int D = tp.D, S = tp.S;
  const Carve L = carve(tp.Dp, S, NT);
  uint16_t *s_goff = reinterpret_cast<uint16_t *>(smem + L.goff);
  float *s_ohp = reinterpret_cast<float *>(smem + L.ohp);
  float *s_rows = reinterpret_cast<float *>(smem + L.rows);
  unsigned char *s_ring = smem + L.ring;
  float *s_red = reinterpret_cast<float *>(smem + L.red);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ntiles = (n + kRows - 1) / kRows;
  load_tables(tp, s_goff, s_ohp);
  // the next tile's rows are requested inside eval_tile (problems without pair terms)
  bool requested = false;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int row0 = tile * kRows;
    __syncthreads();  // the previous tile's readers of the rows are done
    if (!requested) issue_rows(x, row0, n, D, S, s_rows, wide != 0, lane, wave);
    finish_rows(D, S, s_rows);
    const int next = tile + static_cast<int>(gridDim.x);
    const NextRows nx{x, next < ntiles && !tp.any_pairwise ? next * kRows : -1, n, D, wide != 0};
    constexpr int kAheadSteps = (NT == 2 ? 4 : 3) - (MW > kMW ? 1 : 0);
    const float F = eval_tile<NT, KIND, kAheadSteps, false, MW>(tp, s_rows, S, s_goff, s_ohp, s_ring, s_red, lane, wave, nx);
    requested = nx.row0 >= 0;
    if (wave == 0 && lane < kRows && row0 + lane < n) out[row0 + lane] = F + static_cast<float>(tp.bias);
  }
}

// One component of a fused composition: its tiled tables (device copy) and arithmetic.
struct CompDesc {
  TiledProb tp;
  int six;        // split mode: six products
  int unrotated;  // z = s (x - o_hi) + c' per variable, no rotation (no pair terms)
  int index;      // the component's place in the composition (sigma, lambda, bias, G order)
};

// Unrotated component on the staged rows: each wave takes rows, lanes the variables; returns the
// component value in wave 0 lanes < 32 (through s_red).
__device__ __forceinline__ float eval_unrotated(const TiledProb &tp, const float *s_rows, int S, float *s_red, int lane,
                                                int wave) {
  const float s = static_cast<float>(tp.scale0);
  const float *oh = static_cast<const float *>(tp.oh);
  const float *czp = static_cast<const float *>(tp.cz);
  const float *cfp = static_cast<const float *>(tp.coef);
  const TiledSeg &sg = tp.segs[0];
  const float prm = seg_param(sg);
  for (int rr = wave; rr < kRows; rr += kWaves) {
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
  const float F = (wave == 0 && lane < kRows) ? s_red[lane * kSlots] : 0.0f;
  __syncthreads();
  return F;
}

// LDS carve of the fused composition: the row carve for the largest component tables (ring for
// six products), then the component values (FP32) and squared distances (FP64) per
// (component, row).
struct CompCarve {
  Carve base;
  int g, d2, total;
};
__host__ __device__ inline CompCarve comp_carve(int Dpmax, int S) {
  CompCarve c;
  c.base = carve(Dpmax, S, 3);
  c.g = c.base.total;
  c.d2 = c.g + round16(8 * kRows * 4);
  c.total = c.d2 + 8 * kRows * 8;
  return c;
}

// Composition (Sec. 6, Eqs. (composition) and (weight)) with every component on the same staged
// rows: X is read from HBM once.  Per tile: d_i^2 = |x - o^i|^2 in FP64 from the staged FP32 rows
// (before any component writes z over them), then each component's value G_i in the order of
// comps (its gather tables loaded into LDS in turn, f_opt excluded; a component with pair terms,
// which overwrites the rows, comes last), log-domain weights in FP64 (one-hot where some
// d_i = 0), F = sum omega_i (lambda_i G_i + bias_i) + f_opt.
// (A template so that the headers including this one define no kernel symbol of their own.)
template <int NTMAX>
__global__ __launch_bounds__(kThreads) void k_rowres_comp(const CompDesc *__restrict__ comps, int nc, int Dpmax,
                                                          int S, const float *__restrict__ x, int n, int D,
                                                          const double *__restrict__ o64,
                                                          const double *__restrict__ sigma,
                                                          const double *__restrict__ lambda,
                                                          const double *__restrict__ bias, double fopt,
                                                          float *__restrict__ out, int wide) {
  extern __shared__ __align__(16) unsigned char smem[];
  static_assert(NTMAX == 3, "the composition ring holds six-product steps");
  const CompCarve L = comp_carve(Dpmax, S);
  uint16_t *s_goff = reinterpret_cast<uint16_t *>(smem + L.base.goff);
  float *s_ohp = reinterpret_cast<float *>(smem + L.base.ohp);
  float *s_rows = reinterpret_cast<float *>(smem + L.base.rows);
  unsigned char *s_ring = smem + L.base.ring;
  float *s_red = reinterpret_cast<float *>(smem + L.base.red);
  float *s_g = reinterpret_cast<float *>(smem + L.g);
  double *s_d2 = reinterpret_cast<double *>(smem + L.d2);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ntiles = (n + kRows - 1) / kRows;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int row0 = tile * kRows;
    __syncthreads();
    stage_rows(x, row0, n, D, S, s_rows, wide != 0, lane, wave);
    // squared distances to every optimum in FP64 (the FP32 rows widen exactly): each wave takes
    // rows, lanes the variables
    for (int rr = wave; rr < kRows; rr += kWaves) {
      for (int i = 0; i < nc; ++i) {
        double acc = 0.0;
        for (int j = lane; j < D; j += 64) {
          const double d = static_cast<double>(s_rows[rr * S + j]) - o64[static_cast<size_t>(i) * D + j];
          acc += d * d;
        }
#pragma unroll
        for (int sh = 1; sh < 64; sh <<= 1) acc += __shfl_xor(acc, sh, 64);
        if (lane == 0) s_d2[i * kRows + rr] = acc;
      }
    }
    for (int k = 0; k < nc; ++k) {
      const CompDesc &cd = comps[k];
      float G;
      if (cd.unrotated) {
        G = eval_unrotated(cd.tp, s_rows, S, s_red, lane, wave);
      } else {
        __syncthreads();  // the previous component's readers of the tables are done
        load_tables(cd.tp, s_goff, s_ohp);
        __syncthreads();
        const NextRows none{x, -1, n, D, false};
        if (cd.six) G = eval_tile<3, -1, 2, true>(cd.tp, s_rows, S, s_goff, s_ohp, s_ring, s_red, lane, wave, none);
        else G = eval_tile<2, -1, 3, true>(cd.tp, s_rows, S, s_goff, s_ohp, s_ring, s_red, lane, wave, none);
      }
      if (wave == 0 && lane < kRows) s_g[cd.index * kRows + lane] = G;
    }
    __syncthreads();
    if (wave == 0 && lane < kRows && row0 + lane < n) {
      int nzero = 0;
      double amax = -1.0e308;
      for (int i = 0; i < nc; ++i) {
        const double d2 = s_d2[i * kRows + lane];
        if (d2 == 0.0) ++nzero;
        else amax = fmax(amax, -0.5 * log(d2) - d2 / (2.0 * D * sigma[i] * sigma[i]));
      }
      double wsum = 0.0, g = 0.0;
      for (int i = 0; i < nc; ++i) {
        const double d2 = s_d2[i * kRows + lane];
        const double w = nzero ? (d2 == 0.0 ? 1.0 : 0.0)
                               : exp(-0.5 * log(d2) - d2 / (2.0 * D * sigma[i] * sigma[i]) - amax);
        wsum += w;
        g += w * (lambda[i] * static_cast<double>(s_g[i * kRows + lane]) + bias[i]);
      }
      out[row0 + lane] = static_cast<float>(g / wsum + fopt);
    }
  }
}

}  // namespace rowres

}  // namespace curob
