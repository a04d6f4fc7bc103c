// tiled_tables.cpp -- host construction of the tiled path's device tables (basic functions of
// any dimension, hybrid functions of Sec. 5).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "tables.h"
#include "tiled.h"

namespace curob {

void TiledDev::release() {
  for (void *p : allocs) (void)hipFree(p);
  allocs.clear();
  ready = false;
}

namespace {

size_t pad16(size_t b) { return (b + 15) & ~static_cast<size_t>(15); }
int ceil32(int n) { return (n + 31) / 32 * 32; }

struct HostBlock {
  int off;       // first packed position in the problem's own (unpadded) packed order
  int n;         // size
  int seg;       // formula segment
  const std::vector<double> *Q;  // n x n, or nullptr for the identity
  double s;      // scale folded into the tile values
};

}  // namespace

hipError_t build_tiled(const Problem &p, int path, TiledDev &td, std::string &err) {
  td.release();
  if (p.type == Problem::COMPOSITION) {
    err = "compositions are evaluated component by component";
    return hipErrorInvalidValue;
  }
  const bool f64 = path == PATH_F64;
  const size_t esz = f64 ? 8 : 4;
  const int KW = kw_of(path);
  const int D = p.dim;

  // blocks and formula segments
  std::vector<HostBlock> blocks;
  std::vector<int> orig(D);
  const bool hybrid = p.type == Problem::HYBRID;
  const Segment &s0 = p.segs[0];
  const bool rotate = p.rotated && !(!hybrid && s0.base == 0 && s0.c == 0.0);  // sphere: Sec. 3.1 invariance
  if (rotate) {
    for (int j = 0; j < D; ++j) orig[j] = p.orig[j];
    for (size_t k = 0; k < p.Q.size(); ++k)
      blocks.push_back(HostBlock{p.blk_off[k], p.blk_n[k], hybrid ? static_cast<int>(k) : 0, &p.Q[k],
                                 hybrid ? p.segs[k].s : s0.s});
  } else {
    // unrotated: identity blocks of 32 variables in original order
    for (int j = 0; j < D; ++j) orig[j] = j;
    for (int off = 0; off < D; off += 32) blocks.push_back(HostBlock{off, std::min(32, D - off), 0, nullptr, s0.s});
  }
  const int nseg = hybrid ? static_cast<int>(p.segs.size()) : 1;
  if (nseg > kMaxSegments) {
    err = "too many formula segments";
    return hipErrorInvalidValue;
  }

  // padded layout
  std::vector<int> poff(blocks.size());
  int Dp = 0;
  for (size_t b = 0; b < blocks.size(); ++b) {
    poff[b] = Dp;
    Dp += ceil32(blocks[b].n);
  }
  std::vector<int> gidx(Dp, -1), pos_of(D, -1), seg_of_p(Dp, 0), idx_in_seg(Dp, -1);
  for (size_t b = 0; b < blocks.size(); ++b)
    for (int a = 0; a < ceil32(blocks[b].n); ++a) {
      const int pp = poff[b] + a;
      seg_of_p[pp] = blocks[b].seg;
      if (a < blocks[b].n) {
        const int j = orig[blocks[b].off + a];
        gidx[pp] = j;
        pos_of[j] = pp;
        idx_in_seg[pp] = hybrid ? a : j;
      }
    }

  // per padded position tables
  std::vector<unsigned char> oh(pad16(D * esz), 0), cz(pad16(Dp * esz), 0), coef(pad16(Dp * esz), 0);
  auto store = [&](std::vector<unsigned char> &buf, size_t i, double v) {
    if (f64) {
      std::memcpy(buf.data() + i * 8, &v, 8);
    } else {
      const float f = static_cast<float>(v);
      std::memcpy(buf.data() + i * 4, &f, 4);
    }
  };
  std::vector<double> olo(D, 0.0);
  for (int j = 0; j < D; ++j) {
    store(oh, j, p.o[j]);
    if (!f64) olo[j] = p.o[j] - static_cast<double>(static_cast<float>(p.o[j]));
  }
  std::vector<int> succ(Dp, -1);
  for (size_t b = 0; b < blocks.size(); ++b) {
    const HostBlock &B = blocks[b];
    const Segment &sg = p.segs[hybrid ? B.seg : 0];
    const int kind = fn_spec(sg.base).kind;
    for (int a = 0; a < ceil32(B.n); ++a) {
      const int pp = poff[b] + a;
      if (a >= B.n) {
        if (kind == K_POWERS) store(coef, pp, 2.0);
        // z = -1/2 makes every Weierstrass cosine argument exactly 0 (3^k is not exact in FP32)
        if (kind == K_WEIERSTRASS) store(cz, pp, -0.5);
        continue;
      }
      // c' = c - s (Q o_lo) for this output position
      double corr = 0.0;
      for (int c = 0; c < B.n; ++c) {
        const double qv = B.Q ? (*B.Q)[static_cast<size_t>(a) * B.n + c] : (a == c ? 1.0 : 0.0);
        corr += qv * olo[orig[B.off + c]];
      }
      // the family's constant shift of z (Schwefel, HappyCat, HGBat) is folded into c'
      // (padding gives w = 0)
      store(cz, pp, sg.c - B.s * corr + kind_zshift(kind));
      const int n_f = hybrid ? sg.n : D;
      double cf = formula_coef(sg.base, idx_in_seg[pp], n_f);
      if (kind == K_GRIEWANK) cf /= 2.0 * M_PI;  // the cosine takes revolutions
      store(coef, pp, cf);
      if (kind_is_pairwise(kind)) {
        const bool wraps = kind_pair_wraps(kind);
        if (hybrid) {
          const int na = a + 1 < B.n ? a + 1 : (wraps ? 0 : -1);
          succ[pp] = na >= 0 ? poff[b] + na : -1;
        } else {
          const int i = idx_in_seg[pp];
          const int ni = i + 1 < D ? i + 1 : (wraps ? 0 : -1);
          succ[pp] = ni >= 0 ? pos_of[ni] : -1;
        }
      }
    }
  }

  // dense tiles of s*Q per block, and the output groups
  std::vector<int> blk4, grp4;
  std::vector<unsigned char> qfrag;
  int ntiles = 0;
  const int nterm = is_split(path) ? split_terms(path) : 1;
  const size_t tile_bytes = is_split(path) ? static_cast<size_t>(nterm) * 64 * 16 : 64 * esz;
  for (size_t b = 0; b < blocks.size(); ++b) {
    const HostBlock &B = blocks[b];
    const int np = ceil32(B.n);
    const int mt = np / 16, kt = np / KW;
    blk4.insert(blk4.end(), {poff[b], np, ntiles, kt});
    auto qv = [&](int row, int col) -> double {
      if (row >= B.n || col >= B.n) return 0.0;
      const double v = B.Q ? (*B.Q)[static_cast<size_t>(row) * B.n + col] : (row == col ? 1.0 : 0.0);
      return B.s * v;
    };
    qfrag.resize(qfrag.size() + tile_bytes * mt * kt);
    for (int ml = 0; ml < mt; ++ml)
      for (int kl = 0; kl < kt; ++kl) {
        unsigned char *dst = qfrag.data() + static_cast<size_t>(ntiles) * tile_bytes;
        if (is_split(path)) {
          uint16_t *qb = reinterpret_cast<uint16_t *>(dst);
          for (int l = 0; l < 64; ++l)
            for (int e = 0; e < 8; ++e) {
              double rest = qv(16 * ml + l % 16, 32 * kl + 8 * (l / 16) + e);
              for (int term = 0; term < nterm; ++term) {
                const uint16_t h = bf16_bits_rne(static_cast<float>(rest));
                rest -= static_cast<double>(bf16_bits_to_float(h));
                qb[(static_cast<size_t>(term) * 64 + l) * 8 + e] = h;
              }
            }
        } else {
          for (int l = 0; l < 64; ++l) {
            const double v = qv(16 * ml + l % 16, 4 * kl + l / 16);
            if (f64) {
              std::memcpy(dst + l * 8, &v, 8);
            } else {
              const float f = static_cast<float>(v);
              std::memcpy(dst + l * 4, &f, 4);
            }
          }
        }
        ++ntiles;
      }
    for (int m0 = 0; m0 < mt; m0 += kGroupMTiles)
      grp4.insert(grp4.end(), {static_cast<int>(b), m0, std::min(kGroupMTiles, mt - m0), B.seg});
  }
  const int ngroups = static_cast<int>(grp4.size() / 4);

  TiledProb &tp = td.tp;
  tp = TiledProb{};
  // row-resident kernel tables (split paths): byte offset of each padded position's variable
  // within an LDS row, the zero slot at column D for padding, and o_hi in packed order
  std::vector<uint16_t> goff16(Dp, static_cast<uint16_t>(D * 4));
  std::vector<float> ohp(Dp, 0.0f);
  if (!f64 && D * 4 < 65536) {
    for (int pp = 0; pp < Dp; ++pp)
      if (gidx[pp] >= 0) {
        goff16[pp] = static_cast<uint16_t>(gidx[pp] * 4);
        ohp[pp] = static_cast<float>(p.o[gidx[pp]]);
      }
  }
  tp.S = lds_stride(D, 0);
  tp.D = D;
  tp.Dp = Dp;
  tp.nblocks = static_cast<int>(blocks.size());
  tp.ngroups = ngroups;
  tp.nsegs = nseg;
  tp.bias = p.fopt;
  tp.any_pairwise = 0;
  tp.pair_mtiles_max = 0;
  tp.mtiles_max = 0;
  for (size_t b = 0; b < blocks.size(); ++b) {
    tp.mtiles_max = std::max(tp.mtiles_max, ceil32(blocks[b].n) / 16);
    if (kind_is_pairwise(fn_spec(p.segs[hybrid ? blocks[b].seg : 0].base).kind))
      tp.pair_mtiles_max = std::max(tp.pair_mtiles_max, ceil32(blocks[b].n) / 16);
  }
  // unrotated basic problems: the identity blocks of 32 keep packed position = variable, and
  // the row-wise kernel reads the per-position tables by variable
  tp.rowwise = (!hybrid && !rotate) ? 1 : 0;
  tp.scale0 = s0.s;
  for (int sgi = 0; sgi < nseg; ++sgi) {
    const Segment &sg = p.segs[sgi];
    TiledSeg &ts = tp.segs[sgi];
    ts.base = sg.base;
    ts.kind = fn_spec(sg.base).kind;
    ts.n = hybrid ? sg.n : D;
    ts.pairwise = kind_is_pairwise(ts.kind) ? 1 : 0;
    tp.any_pairwise |= ts.pairwise;
    ts.kparam = 10.0 / std::pow(static_cast<double>(ts.n), 1.2);
    ts.g0 = ngroups;
    ts.g1 = 0;
    for (int g = 0; g < ngroups; ++g)
      if (grp4[4 * g + 3] == sgi) {
        ts.g0 = std::min(ts.g0, g);
        ts.g1 = std::max(ts.g1, g + 1);
      }
    ts.p0 = Dp;
    ts.p1 = 0;
    int npad = 0;
    for (int pp = 0; pp < Dp; ++pp)
      if (seg_of_p[pp] == sgi) {
        ts.p0 = std::min(ts.p0, pp);
        ts.p1 = std::max(ts.p1, pp + 1);
        if (gidx[pp] < 0) ++npad;
      }
    ts.padc[0] = ts.padc[1] = ts.padc[2] = 0.0;
    if (ts.kind == K_WEIERSTRASS) ts.padc[0] = npad * (2.0 - 9.5367431640625e-07);
    if (ts.kind == K_ACKLEY) ts.padc[1] = npad;
    if (ts.kind == K_HGBAT) ts.padc[1] = 2.0 * npad;
    if (ts.kind == K_SCHWEFEL) ts.padc[0] = npad * schwefel_pad_term(f64);
    if (ts.kind == K_LUNACEK) {
      ts.padc[0] = 6.25 * npad;
      ts.padc[1] = 6.25 * npad;
      ts.padc[2] = -npad;
    }
  }

  auto up = [&](const void *src, size_t bytes, const void **dst) -> hipError_t {
    void *d = nullptr;
    hipError_t e = hipMalloc(&d, pad16(bytes > 0 ? bytes : 16));
    if (e != hipSuccess) return e;
    td.allocs.push_back(d);
    if (bytes) e = hipMemcpy(d, src, bytes, hipMemcpyHostToDevice);
    *dst = d;
    return e;
  };
  hipError_t e;
  if ((e = up(gidx.data(), gidx.size() * 4, reinterpret_cast<const void **>(&tp.gidx))) != hipSuccess) return e;
  if ((e = up(oh.data(), oh.size(), &tp.oh)) != hipSuccess) return e;
  if ((e = up(cz.data(), cz.size(), &tp.cz)) != hipSuccess) return e;
  if ((e = up(coef.data(), coef.size(), &tp.coef)) != hipSuccess) return e;
  if ((e = up(succ.data(), succ.size() * 4, reinterpret_cast<const void **>(&tp.succ))) != hipSuccess) return e;
  if ((e = up(qfrag.data(), qfrag.size(), &tp.qfrag)) != hipSuccess) return e;
  tp.qfrag_kib = static_cast<int>((qfrag.size() + 1023) / 1024);
  if ((e = up(blk4.data(), blk4.size() * 4, reinterpret_cast<const void **>(&tp.blocks))) != hipSuccess) return e;
  if ((e = up(grp4.data(), grp4.size() * 4, reinterpret_cast<const void **>(&tp.groups))) != hipSuccess) return e;
  if ((e = up(goff16.data(), goff16.size() * 2, reinterpret_cast<const void **>(&tp.goff))) != hipSuccess) return e;
  if ((e = up(ohp.data(), ohp.size() * 4, reinterpret_cast<const void **>(&tp.ohp))) != hipSuccess) return e;
  td.ready = true;
  return hipSuccess;
}

size_t tiled_partials_bytes(const TiledProb &tp, int path, int rows) {
  const size_t esz = path == PATH_F64 ? 8 : 4;
  return tp.rowwise ? 0 : static_cast<size_t>(tp.ngroups) * rows * kPartialSlots * esz;
}

size_t tiled_pack_bytes(const TiledProb &tp, int path, int rows) {
  const size_t bpp = is_split(path) ? 2 * split_terms(path) : (path == PATH_F64 ? 8 : 4);
  return tp.rowwise ? 0 : static_cast<size_t>(rows) * tp.Dp * bpp;
}

size_t tiled_z_bytes(const TiledProb &tp, int path, int rows) {
  const size_t esz = path == PATH_F64 ? 8 : 4;
  return tp.any_pairwise && !tp.rowwise ? static_cast<size_t>(rows) * tp.Dp * esz : 0;
}

}  // namespace curob
