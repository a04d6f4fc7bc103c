// tables.cpp -- per-problem device tables for the resident evaluation kernel.
//
// Variables are renumbered into "packed" order: the three random groups of Sec. 1.2 one after
// another, so the rotation becomes block diagonal.  The kernel multiplies by the packed matrix
// (pre-scaled by the function's s) tile by tile, skipping tiles that are all zero.
#include "tables.h"

#include <algorithm>
#include <cmath>
#include <cstring>

#include "kernels.h"
#include "problem.h"
#include "schwefel_series.h"

namespace curob {

void DevTables::release() {
  for (void *p : allocs) (void)hipFree(p);
  allocs.clear();
  ready = false;
}

uint16_t bf16_bits_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

float bf16_bits_to_float(uint16_t h) {
  uint32_t u = static_cast<uint32_t>(h) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

double schwefel_pad_term(bool f64) {
  if (!f64) return static_cast<double>(kSchwefelT0);
  return kSchwefelC - kSchwefelW * std::sin(std::sqrt(kSchwefelW));
}

int lds_stride(int D, int m) {
  const int need = D + 1 > m ? D + 1 : m;
  int u = (need + 3) / 4;
  if ((u & 1) == 0) ++u;
  return 4 * u;
}

namespace {

template <typename T>
void put(std::vector<unsigned char> &buf, size_t i, T v) {
  std::memcpy(buf.data() + i * sizeof(T), &v, sizeof(T));
}

size_t pad16(size_t b) { return (b + 15) & ~static_cast<size_t>(15); }

// Order of the variables within each rotation block (any order works: the block is permuted
// on both sides) chosen for the LDS banks.  Each gather instruction of the split paths reads,
// for 16 rows whose LDS stride is 4 (mod 8) words, the packed positions 32 kt + 8 q + e of
// the four lane groups q; the 64 reads fall in distinct banks (or in pairs, with 32 banks)
// exactly when the four variables differ mod 4.  Pairwise families also read the z of the
// successors of positions 16 m + 4 q + e, under the same condition on the successors' packed
// positions.  A deterministic local search over swaps within a block minimises the number of
// repeated residues.  loc maps packed position -> index into the problem's packed order.
void balance_banks(const Problem &p, int D, int KT, int MT, bool pair, bool wraps, std::vector<int> &loc) {
  const int nb = static_cast<int>(p.blk_off.size());
  std::vector<int> order(D), slot(D);
  auto cost = [&]() {
    for (int pp = 0; pp < D; ++pp) {
      order[pp] = p.orig[loc[pp]];
      slot[order[pp]] = pp;
    }
    int c = 0;
    for (int kt = 0; kt < KT; ++kt)
      for (int e = 0; e < 8; ++e) {
        unsigned mask = 0;
        for (int q = 0; q < 4; ++q) {
          const int pp = 32 * kt + 8 * q + e;
          mask |= 1u << ((pp < D ? order[pp] : D) & 3);
        }
        c += 4 - __builtin_popcount(mask);
      }
    if (pair) {
      for (int m = 0; m < MT; ++m)
        for (int e = 0; e < 4; ++e) {
          unsigned mask = 0;
          for (int q = 0; q < 4; ++q) {
            const int pp = 16 * m + 4 * q + e;
            int sp = pp;
            if (pp < D) {
              const int ni = order[pp] + 1 < D ? order[pp] + 1 : (wraps ? 0 : -1);
              if (ni >= 0) sp = slot[ni];
            }
            mask |= 1u << (sp & 3);
          }
          c += 4 - __builtin_popcount(mask);
        }
    }
    return c;
  };
  int best = cost();
  uint64_t st = 0x9E3779B97F4A7C15ULL ^ static_cast<uint64_t>(D);
  auto next = [&]() {
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    return st;
  };
  for (int it = 0; it < 3000 && best > 0; ++it) {
    const int k = static_cast<int>(next() % static_cast<uint64_t>(nb));
    const int n = p.blk_n[k];
    if (n < 2) continue;
    const int a = p.blk_off[k] + static_cast<int>(next() % static_cast<uint64_t>(n));
    const int b = p.blk_off[k] + static_cast<int>(next() % static_cast<uint64_t>(n));
    if (a == b) continue;
    std::swap(loc[a], loc[b]);
    const int c = cost();
    if (c <= best) best = c;
    else std::swap(loc[a], loc[b]);
  }
}

}  // namespace

bool build_host_tables(const Problem &p, int path, HostTables &ht, std::string &err) {
  if (p.type != Problem::BASIC) {
    err = "hybrid and composition problems use the composite kernels";
    return false;
  }
  const int D = p.dim;
  if (D > 16 * kMaxMT) {
    err = "resident kernel supports dimension <= 128";
    return false;
  }
  const bool f64 = path == PATH_F64;
  const size_t esz = f64 ? 8 : 4;
  const int KW = kw_of(path);
  const int KT = (D + KW - 1) / KW;
  const int MT = (D + 15) / 16;
  const int Mp = 16 * MT;
  const Segment &seg = p.segs[0];
  const int base = seg.base;
  const int kind = fn_spec(base).kind;
  const double s = seg.s, c = seg.c;

  ht = HostTables{};
  ht.path = path;
  auto store = [&](std::vector<unsigned char> &buf, size_t i, double v) {
    if (f64) put<double>(buf, i, v); else put<float>(buf, i, static_cast<float>(v));
  };
  // The sphere is rotation invariant (Sec. 3.1): |R y|^2 = |y|^2, so it is evaluated without
  // the rotation, in original variable order.
  const bool rotate = p.rotated && !(base == 0 && c == 0.0);
  const bool pair = kind_is_pairwise(kind), wraps = kind_pair_wraps(kind);
  // packed position -> index into the problem's packed order: the identity, or on the rotated
  // split paths a permutation within each block chosen for the LDS banks
  std::vector<int> loc(D);
  for (int pp = 0; pp < D; ++pp) loc[pp] = pp;
  if (rotate && is_split(path)) balance_banks(p, D, KT, MT, pair, wraps, loc);
  std::vector<int> order(D), slot(D);
  for (int pp = 0; pp < D; ++pp) {
    order[pp] = rotate ? p.orig[loc[pp]] : pp;
    slot[order[pp]] = pp;
  }
  // shift: the path's rounding o_hi, and (FP32 paths) the remainder o_lo = o - o_hi.  The
  // split paths subtract o_hi while gathering the packed operand, so they keep it in packed
  // order (zeros past D); the other paths subtract it in original order while staging rows.
  std::vector<double> olo(D, 0.0);
  const bool split = is_split(path);
  ht.oh.assign(pad16(static_cast<size_t>(split ? std::max(D, std::max(KT * KW, Mp)) : D) * esz), 0);
  for (int j = 0; j < D; ++j) {
    if (!f64) olo[j] = p.o[j] - static_cast<double>(static_cast<float>(p.o[j]));
  }
  for (int pp = 0; pp < D; ++pp) store(ht.oh, pp, p.o[split ? order[pp] : pp]);
  // packed block-diagonal rotation, scaled by s
  const int nb = static_cast<int>(p.Q.size());
  auto qp = [&](int row, int col) -> double {
    if (!rotate || row >= D || col >= D) return 0.0;
    row = loc[row];
    col = loc[col];
    for (int k = 0; k < nb; ++k) {
      const int off = p.blk_off[k], n = p.blk_n[k];
      if (row >= off && row < off + n) {
        if (col >= off && col < off + n) return s * p.Q[k][static_cast<size_t>(row - off) * n + (col - off)];
        return 0.0;
      }
    }
    return 0.0;
  };
  // gather: byte offset of each packed position's variable within an LDS row; padding reads
  // the zero slot at column D
  ht.goff.assign(pad16(KT * KW * 2) / 2, static_cast<uint16_t>(D * esz));
  for (int pp = 0; pp < D; ++pp) ht.goff[pp] = static_cast<uint16_t>(order[pp] * esz);
  // per packed position: c' = c - s (Q o_lo)_p, coefficient, formula successor.  Padding gets
  // z = 0 (Weierstrass: -1/2) and neutral coefficients.  The family's constant shift of z
  // (Schwefel's 420.9687..., HappyCat's and HGBat's 1) is folded into c'; their padding gives w = 0.
  ht.cz.assign(pad16(Mp * esz), 0);
  ht.coef.assign(pad16(Mp * esz), 0);
  ht.succ.assign(pad16(Mp * 2) / 2, static_cast<int16_t>(-1));
  for (int pp = 0; pp < Mp; ++pp) {
    if (pp >= D) {
      if (kind == K_POWERS) store(ht.coef, pp, 2.0);
      // Weierstrass padding takes z = -1/2, so every cosine argument 2 pi 3^k (z + 1/2) is
      // exactly 0 in any precision (3^k itself is not exact in FP32 beyond k = 15)
      if (kind == K_WEIERSTRASS) store(ht.cz, pp, -0.5);
      continue;
    }
    const int i = order[pp];  // index the formula sees (original variable order)
    double corr;
    if (rotate) {
      corr = 0.0;
      for (int qq = 0; qq < D; ++qq) corr += qp(pp, qq) * olo[order[qq]];
    } else {
      corr = s * olo[i];
    }
    store(ht.cz, pp, c - corr + kind_zshift(kind));
    double cf = formula_coef(base, i, D);
    if (kind == K_GRIEWANK) cf /= 2.0 * M_PI;  // the cosine takes revolutions
    store(ht.coef, pp, cf);
    if (pair) {
      const int ni = i + 1 < D ? i + 1 : (wraps ? 0 : -1);
      ht.succ[pp] = static_cast<int16_t>(ni >= 0 ? slot[ni] : -1);
    }
  }
  // nonzero tiles of s * Qp, m-tile by m-tile: the rows 16 m .. 16 m + 15 meet the blocks
  // whose columns span a contiguous k-tile range
  int ntiles = 0;
  ht.mtab.assign(4 * MT, 0);
  if (rotate) {
    std::vector<std::pair<int, int>> tiles;  // (m, kt)
    for (int m = 0; m < MT; ++m) {
      const int r0 = 16 * m, r1 = std::min(D, r0 + 16) - 1;
      int klo = 1 << 30, khi = -1;
      for (int k = 0; k < nb; ++k) {
        const int off = p.blk_off[k], n = p.blk_n[k];
        if (off <= r1 && off + n - 1 >= r0) {
          klo = std::min(klo, off / KW);
          khi = std::max(khi, (off + n - 1) / KW);
        }
      }
      ht.mtab[4 * m + 0] = klo;
      ht.mtab[4 * m + 1] = khi;
      ht.mtab[4 * m + 2] = static_cast<int>(tiles.size());
      // split paths (k-tiles of 32, at most four): the range as one dispatch code
      if (is_split(path)) ht.mtab[4 * m + 3] = 4 * klo + (khi - klo);
      for (int kt = klo; kt <= khi; ++kt) tiles.emplace_back(m, kt);
    }
    ntiles = static_cast<int>(tiles.size());
    if (is_split(path)) {
      // tile t: nterm fragments [64 lanes][8] (hi, [mid,] lo); lane l holds
      // A[i = l % 16][k = 8 (l / 16) + e] = s Qp[16 m + i][32 kt + k], split into bf16 terms
      const int nterm = split_terms(path);
      ht.qfrag.assign(static_cast<size_t>(ntiles) * nterm * 64 * 8 * 2, 0);
      uint16_t *qb = reinterpret_cast<uint16_t *>(ht.qfrag.data());
      for (int t = 0; t < ntiles; ++t) {
        const int m = tiles[t].first, kt = tiles[t].second;
        for (int l = 0; l < 64; ++l)
          for (int e = 0; e < 8; ++e) {
            double rest = qp(16 * m + l % 16, 32 * kt + 8 * (l / 16) + e);
            for (int term = 0; term < nterm; ++term) {
              const uint16_t b = bf16_bits_rne(static_cast<float>(rest));
              rest -= static_cast<double>(bf16_bits_to_float(b));
              qb[((static_cast<size_t>(t) * nterm + term) * 64 + l) * 8 + e] = b;
            }
          }
      }
    } else {
      // tile t: [64 lanes], lane l holds A[i = l % 16][k = l / 16] = s Qp[16 m + i][4 kt + k]
      ht.qfrag.assign(pad16(static_cast<size_t>(ntiles) * 64 * esz), 0);
      for (int t = 0; t < ntiles; ++t) {
        const int m = tiles[t].first, kt = tiles[t].second;
        for (int l = 0; l < 64; ++l) store(ht.qfrag, static_cast<size_t>(t) * 64 + l, qp(16 * m + l % 16, 4 * kt + l / 16));
      }
    }
  }

  DevProb &pb = ht.pb;
  pb.D = D;
  // the unrotated read-out and the pairwise z exchange reach position 16 MT - 1 of a row; rows
  // loaded directly are only gathered from (positions < D and the zero slot at D)
  pb.S = lds_stride(D, direct_rows(path, rotate ? 1 : 0, kind) ? 0 : Mp);
  pb.KT = KT;
  pb.MT = MT;
  pb.ntiles = ntiles;
  pb.rotated = rotate ? 1 : 0;
  pb.kind = kind;
  pb.Df = D;
  pb.bias = p.fopt;
  pb.kparam = 10.0 / std::pow(static_cast<double>(D), 1.2);
  pb.scale = s;
  // what the padded positions (z = 0, or w = 0 for the shifted families) add to each sum
  const double npad = static_cast<double>(Mp - D);
  pb.padc[0] = pb.padc[1] = pb.padc[2] = 0.0;
  if (kind == K_WEIERSTRASS) pb.padc[0] = npad * (2.0 - 9.5367431640625e-07);   // sum_k a^k cos(0)
  if (kind == K_ACKLEY) pb.padc[1] = npad;                                          // cos(0) = 1
  if (kind == K_HGBAT) pb.padc[1] = 2.0 * npad;                                     // (0 - 1)(0 - 2)
  if (kind == K_SCHWEFEL) pb.padc[0] = npad * schwefel_pad_term(f64);  // z = 0: the term at the optimum
  if (kind == K_LUNACEK) {
    pb.padc[0] = 6.25 * npad;  // (0 - 2.5)^2
    pb.padc[1] = 6.25 * npad;  // (0 + 2.5)^2
    pb.padc[2] = -npad;        // cos(2 pi (0 - 2.5)) = -1
  }
  return true;
}

hipError_t upload_tables(const HostTables &ht, DevTables &dt) {
  dt.release();
  auto up = [&](const void *src, size_t bytes, const void **dst) -> hipError_t {
    if (bytes == 0) {
      *dst = nullptr;
      return hipSuccess;
    }
    void *d = nullptr;
    hipError_t e = hipMalloc(&d, pad16(bytes));
    if (e != hipSuccess) return e;
    dt.allocs.push_back(d);
    e = hipMemcpy(d, src, bytes, hipMemcpyHostToDevice);
    *dst = d;
    return e;
  };
  // one block in the kernel's LDS order: the setup copies it with a single pass
  DevProb pb = ht.pb;
  const LdsLayout L = lds_layout(ht.path, pb, 1);
  std::vector<unsigned char> img(static_cast<size_t>(L.fixed), 0);
  auto place = [&](int off, int cap, const void *src, size_t bytes) {
    if (cap > 0 && bytes > 0) std::memcpy(img.data() + off, src, std::min(bytes, static_cast<size_t>(cap)));
  };
  place(L.q, L.q_bytes, ht.qfrag.data(), ht.qfrag.size());
  place(L.goff, L.goff_bytes, ht.goff.data(), ht.goff.size() * 2);
  place(L.oh, L.vec_bytes, ht.oh.data(), ht.oh.size());
  place(L.cz, L.mp_bytes, ht.cz.data(), ht.cz.size());
  place(L.coef, L.mp_bytes, ht.coef.data(), ht.coef.size());
  place(L.succ, L.succ_bytes, ht.succ.data(), ht.succ.size() * 2);
  place(L.mtab, L.mtab_bytes, ht.mtab.data(), ht.mtab.size() * 4);
  hipError_t e = up(img.data(), img.size(), &pb.image);
  if (e != hipSuccess) return e;
  pb.image_bytes = L.fixed;
  dt.pb = pb;
  dt.ready = true;
  return hipSuccess;
}

}  // namespace curob
