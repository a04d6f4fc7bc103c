// tables.cpp -- per-problem device tables for the resident evaluation kernel.
//
// Variables are renumbered into "packed" order: the three random groups of Sec. 1.2 (or the
// hybrid groups of Sec. 5) one after another, so the rotation becomes block diagonal.  The
// kernel multiplies by the packed matrix Qp tile by tile, skipping tiles that are all zero.
#include "tables.h"

#include <cmath>
#include <cstring>

#include "kernels.h"

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

int lds_stride(int D) {
  int u = (D + 1 + 3) / 4;
  if ((u & 1) == 0) ++u;
  return 4 * u;
}

namespace {

template <typename T>
void put(std::vector<unsigned char> &buf, size_t i, T v) {
  std::memcpy(buf.data() + i * sizeof(T), &v, sizeof(T));
}

size_t pad16(size_t b) { return (b + 15) & ~static_cast<size_t>(15); }

}  // namespace

bool build_host_tables(const Problem &p, int path, HostTables &ht, std::string &err) {
  if (p.type == Problem::COMPOSITION) {
    err = "composition problems are evaluated component by component";
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
  if (p.type == Problem::HYBRID) {
    err = "hybrid problems use the segmented kernel";
    return false;
  }

  ht = HostTables{};
  ht.path = path;
  auto store = [&](std::vector<unsigned char> &buf, size_t i, double v) {
    if (f64) put<double>(buf, i, v); else put<float>(buf, i, static_cast<float>(v));
  };
  // per original variable: shift and scale
  ht.o.assign(pad16(D * esz), 0);
  ht.olo.assign(f64 ? 0 : pad16(D * esz), 0);
  ht.sj.assign(pad16(D * esz), 0);
  for (int j = 0; j < D; ++j) {
    store(ht.o, j, p.o[j]);
    if (!f64) put<float>(ht.olo, j, static_cast<float>(p.o[j] - static_cast<double>(static_cast<float>(p.o[j]))));
    store(ht.sj, j, seg.s);
  }
  // The sphere is rotation invariant (Sec. 3.1): |R y|^2 = |y|^2, so it is evaluated without
  // the rotation, in original variable order.
  const bool rotate = p.rotated && !(base == 0 && seg.c == 0.0);
  std::vector<int> order(D);
  for (int pp = 0; pp < D; ++pp) order[pp] = rotate ? p.orig[pp] : pp;
  // packed position -> original variable, padding -> D (a zero slot in LDS)
  std::vector<int> slot(D);
  ht.orig.assign(pad16(KT * KW * 2) / 2, static_cast<uint16_t>(D));
  for (int pp = 0; pp < D; ++pp) {
    ht.orig[pp] = static_cast<uint16_t>(order[pp]);
    slot[order[pp]] = pp;
  }
  // per packed position: coefficient, post-offset, formula successor
  ht.coef.assign(pad16(Mp * esz), 0);
  ht.cz.assign(pad16(Mp * esz), 0);
  ht.succ.assign(pad16(Mp * 2) / 2, static_cast<int16_t>(-1));
  const bool pair = kind_is_pairwise(kind), wraps = kind_pair_wraps(kind);
  for (int pp = 0; pp < D; ++pp) {
    const int i = order[pp];  // index the formula sees (original variable order)
    double cf = formula_coef(base, i, D);
    if (kind == K_GRIEWANK && !f64) cf /= 2.0 * M_PI;  // FP32 cosine takes revolutions
    store(ht.coef, pp, cf);
    store(ht.cz, pp, seg.c);
    if (pair) {
      int ni = i + 1 < D ? i + 1 : (wraps ? 0 : -1);
      ht.succ[pp] = static_cast<int16_t>(ni >= 0 ? slot[ni] : -1);
    }
  }
  // nonzero tiles of the packed block-diagonal rotation
  int ntiles = 0;
  ht.ktab.assign(4 * KT, 0);
  if (rotate) {
    const int nb = static_cast<int>(p.Q.size());
    auto qp = [&](int row, int col) -> double {
      if (row >= D || col >= D) return 0.0;
      for (int k = 0; k < nb; ++k) {
        const int off = p.blk_off[k], n = p.blk_n[k];
        if (row >= off && row < off + n) {
          if (col >= off && col < off + n) return p.Q[k][static_cast<size_t>(row - off) * n + (col - off)];
          return 0.0;
        }
      }
      return 0.0;
    };
    std::vector<std::pair<int, int>> tiles;  // (m, kt)
    for (int kt = 0; kt < KT; ++kt) {
      const int c0 = kt * KW, c1 = std::min(D, c0 + KW) - 1;
      int mlo = 1 << 30, mhi = -1;
      for (int k = 0; k < nb; ++k) {
        const int off = p.blk_off[k], n = p.blk_n[k];
        if (off <= c1 && off + n - 1 >= c0) {
          mlo = std::min(mlo, off / 16);
          mhi = std::max(mhi, (off + n - 1) / 16);
        }
      }
      ht.ktab[4 * kt + 0] = mlo;
      ht.ktab[4 * kt + 1] = mhi;
      ht.ktab[4 * kt + 2] = static_cast<int>(tiles.size());
      for (int m = mlo; m <= mhi; ++m) tiles.emplace_back(m, kt);
    }
    ntiles = static_cast<int>(tiles.size());
    if (is_split(path)) {
      // tile t: nterm fragments [64 lanes][8] (hi, [mid,] lo); lane l holds
      // A[i = l % 16][k = 8 (l / 16) + e] = Qp[16 m + i][32 kt + k], split into bf16 terms
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
      // tile t: [64 lanes], lane l holds A[i = l % 16][k = l / 16] = Qp[16 m + i][4 kt + k]
      ht.qfrag.assign(pad16(static_cast<size_t>(ntiles) * 64 * esz), 0);
      for (int t = 0; t < ntiles; ++t) {
        const int m = tiles[t].first, kt = tiles[t].second;
        for (int l = 0; l < 64; ++l) store(ht.qfrag, static_cast<size_t>(t) * 64 + l, qp(16 * m + l % 16, 4 * kt + l / 16));
      }
    }
  }

  DevProb &pb = ht.pb;
  pb.D = D;
  pb.S = lds_stride(D);
  pb.KT = KT;
  pb.MT = MT;
  pb.ntiles = ntiles;
  pb.rotated = rotate ? 1 : 0;
  pb.kind = kind;
  pb.Df = D;
  pb.bias = p.fopt;
  pb.kparam = 10.0 / std::pow(static_cast<double>(D), 1.2);
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
  DevProb pb = ht.pb;
  hipError_t e;
  if ((e = up(ht.o.data(), ht.o.size(), &pb.o)) != hipSuccess) return e;
  if ((e = up(ht.olo.data(), ht.olo.size(), &pb.olo)) != hipSuccess) return e;
  if ((e = up(ht.sj.data(), ht.sj.size(), &pb.sj)) != hipSuccess) return e;
  if ((e = up(ht.orig.data(), ht.orig.size() * 2, reinterpret_cast<const void **>(&pb.orig))) != hipSuccess) return e;
  if ((e = up(ht.coef.data(), ht.coef.size(), &pb.coef)) != hipSuccess) return e;
  if ((e = up(ht.cz.data(), ht.cz.size(), &pb.cz)) != hipSuccess) return e;
  if ((e = up(ht.succ.data(), ht.succ.size() * 2, reinterpret_cast<const void **>(&pb.succ))) != hipSuccess) return e;
  if ((e = up(ht.qfrag.data(), ht.qfrag.size(), &pb.qfrag)) != hipSuccess) return e;
  if ((e = up(ht.ktab.data(), ht.ktab.size() * 4, reinterpret_cast<const void **>(&pb.ktab))) != hipSuccess) return e;
  dt.pb = pb;
  dt.ready = true;
  return hipSuccess;
}

}  // namespace curob
