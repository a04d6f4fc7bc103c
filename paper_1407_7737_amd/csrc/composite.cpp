// composite.cpp -- host side of the tiled path (large-dimension basic functions, hybrids) and
// of compositions.
#include "composite.h"

#include <algorithm>

#include "eval_rowres.h"
#include "kernels.h"

namespace curob {

hipError_t launch_tiled_split(int, const TiledProb &, const void *, void *, int, int, void *, void *, void *,
                              hipStream_t);
hipError_t launch_tiled_split6(int, const TiledProb &, const void *, void *, int, int, void *, void *, void *,
                               hipStream_t);
hipError_t launch_tiled_f32(int, const TiledProb &, const void *, void *, int, int, void *, void *, void *, hipStream_t);
hipError_t launch_tiled_f64(int, const TiledProb &, const void *, void *, int, int, void *, void *, void *, hipStream_t);
hipError_t launch_rowres_split(int, const TiledProb &, const void *, void *, int, int, hipStream_t);
hipError_t launch_rowres_split6(int, const TiledProb &, const void *, void *, int, int, hipStream_t);
hipError_t launch_rowres_comp(const void *desc, int nc, int Dpmax, int S, const float *x, int n, int D,
                              const double *o64, const double *sig, const double *lam, const double *cb, double fopt,
                              float *out, int num_cu, hipStream_t st);
hipError_t launch_blend(bool f64, const void *x, int n, int D, int nc, const double *o, const double *sigma,
                        const double *lambda, const double *bias, const void *G, int gstride, double fopt, void *out,
                        hipStream_t st);

hipError_t launch_tiled(int path, int kind_hint, const TiledProb &tp, const void *x, void *out, int n, int cap,
                        void *partials, void *zbuf, void *pack, hipStream_t st) {
  switch (path) {
    case PATH_SPLIT: return launch_tiled_split(kind_hint, tp, x, out, n, cap, partials, zbuf, pack, st);
    case PATH_SPLIT6: return launch_tiled_split6(kind_hint, tp, x, out, n, cap, partials, zbuf, pack, st);
    case PATH_F32: return launch_tiled_f32(kind_hint, tp, x, out, n, cap, partials, zbuf, pack, st);
    case PATH_F64: return launch_tiled_f64(kind_hint, tp, x, out, n, cap, partials, zbuf, pack, st);
    default: return hipErrorInvalidValue;
  }
}

bool rowres_fits(const TiledProb &tp, int path) {
  if (!is_split(path) || tp.rowwise || tp.goff == nullptr || tp.D > rowres::kMaxD) return false;
  // a block with pair terms writes its z over the rows: it must finish in one pass
  if (tp.pair_mtiles_max > rowres::kPassMTiles) return false;
  return rowres::carve(tp.Dp, tp.S, split_terms(path)).total <= kMaxLdsBytes;
}

hipError_t launch_rowres(int path, int kind_hint, const TiledProb &tp, const void *x, void *out, int n, int num_cu,
                         hipStream_t st) {
  switch (path) {
    case PATH_SPLIT: return launch_rowres_split(kind_hint, tp, x, out, n, num_cu, st);
    case PATH_SPLIT6: return launch_rowres_split6(kind_hint, tp, x, out, n, num_cu, st);
    default: return hipErrorInvalidValue;
  }
}

void CompositeDev::release() {
  for (auto &t : tiled) t.release();
  for (auto &c : comps) {
    for (auto &t : c.tiled) t.release();
    for (auto &r : c.res) r.release();
  }
  comps.clear();
  for (void *p : allocs) (void)hipFree(p);
  allocs.clear();
  ready = false;
}

hipError_t CompositeScratch::reserve(size_t pb, size_t zb, size_t gb, size_t kb) {
  auto grow = [](void *&ptr, size_t &have, size_t want) -> hipError_t {
    if (want <= have) return hipSuccess;
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    have = 0;
    hipError_t e = hipMalloc(&ptr, want);
    if (e == hipSuccess) have = want;
    return e;
  };
  hipError_t e = grow(partials, partials_bytes, pb);
  if (e == hipSuccess) e = grow(zbuf, zbuf_bytes, zb);
  if (e == hipSuccess) e = grow(gbuf, gbuf_bytes, gb);
  if (e == hipSuccess) e = grow(pack, pack_bytes, kb);
  return e;
}

void CompositeScratch::release() {
  if (partials) (void)hipFree(partials);
  if (zbuf) (void)hipFree(zbuf);
  if (gbuf) (void)hipFree(gbuf);
  if (pack) (void)hipFree(pack);
  *this = CompositeScratch{};
}

namespace {

bool fits_resident(const Problem &p) { return p.type == Problem::BASIC && p.dim <= 16 * kMaxMT; }

hipError_t build_basic_or_hybrid(const Problem &p, TiledDev (&tiled)[PATH_COUNT], std::string &err) {
  for (int path = 0; path < PATH_COUNT; ++path) {
    hipError_t e = build_tiled(p, path, tiled[path], err);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t build_composite(const Problem &p, CompositeDev &cd, std::string &err) {
  cd.release();
  cd.dim = p.dim;
  cd.fopt = p.fopt;
  if (p.type == Problem::BASIC) {
    if (fits_resident(p)) return hipSuccess;  // the resident kernel covers it
    cd.kind_hint = fn_spec(p.segs[0].base).kind;
    hipError_t e = build_basic_or_hybrid(p, cd.tiled, err);
    if (e == hipSuccess) cd.ready = true;
    return e;
  }
  if (p.type == Problem::HYBRID) {
    cd.kind_hint = -1;
    hipError_t e = build_basic_or_hybrid(p, cd.tiled, err);
    if (e == hipSuccess) cd.ready = true;
    return e;
  }
  // composition: components with f_opt 0 (G_i excludes it), FP64 blend tables
  cd.is_composition = true;
  const int nc = static_cast<int>(p.comps.size());
  if (nc < 1 || nc > 8) {
    err = "compositions take 1..8 components";
    return hipErrorInvalidValue;
  }
  cd.comps.resize(nc);
  std::vector<double> o(static_cast<size_t>(nc) * p.dim);
  for (int i = 0; i < nc; ++i) {
    Problem c = p.comps[i];
    c.fopt = 0.0;
    std::copy(c.o.begin(), c.o.end(), o.begin() + static_cast<size_t>(i) * p.dim);
    CompositeDev::Component &cc = cd.comps[i];
    cc.six = problem_needs_six(c);
    cc.hybrid = c.type == Problem::HYBRID;
    if (fits_resident(c)) {
      cc.resident = true;
      for (int path = 0; path < PATH_COUNT; ++path) {
        HostTables ht;
        if (!build_host_tables(c, path, ht, err)) return hipErrorInvalidValue;
        hipError_t e = upload_tables(ht, cc.res[path]);
        if (e != hipSuccess) return e;
      }
    } else {
      hipError_t e = build_basic_or_hybrid(c, cc.tiled, err);
      if (e != hipSuccess) return e;
    }
  }
  auto up = [&](const std::vector<double> &v, const double **dst) -> hipError_t {
    void *d = nullptr;
    hipError_t e = hipMalloc(&d, v.size() * sizeof(double));
    if (e != hipSuccess) return e;
    cd.allocs.push_back(d);
    *dst = static_cast<const double *>(d);
    return hipMemcpy(d, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice);
  };
  hipError_t e;
  if ((e = up(o, &cd.o64)) != hipSuccess) return e;
  if ((e = up(p.sigma, &cd.sig)) != hipSuccess) return e;
  if ((e = up(p.lambda, &cd.lam)) != hipSuccess) return e;
  if ((e = up(p.cbias, &cd.cb)) != hipSuccess) return e;
  // the fused composition kernel: every component above the resident range, rotated ones on the
  // row-resident kernel, unrotated ones without pair terms, at most one component with pair
  // terms (its z overwrites the staged rows, so it runs last), and the rotation tiles of all
  // components together small enough to stay in a die's L2 (4 MiB) next to the streaming rows.
  // Every row tile of the fused kernel walks all components, so larger tile sets would go back
  // to the MALL on every tile; separate launches then keep one component's tiles in L2 at a time
  // and re-read X instead (D = 1000, eight components: 0.56 ms separate, 0.82 ms fused).
  constexpr int kFusedTileKiB = 2048;
  bool fused = p.dim <= rowres::kMaxD;
  int dpmax = 0, npairs = 0, tile_kib = 0;
  for (const auto &cc : cd.comps) {
    if (cc.resident) {
      fused = false;
      break;
    }
    npairs += cc.tiled[PATH_SPLIT].tp.any_pairwise ? 1 : 0;
    for (int path : {PATH_SPLIT, PATH_SPLIT6}) {
      const TiledProb &tp = cc.tiled[path].tp;
      if (tp.rowwise) {
        if (tp.any_pairwise) fused = false;
      } else {
        if (!rowres_fits(tp, path)) fused = false;
        dpmax = std::max(dpmax, tp.Dp);
        if (path == (cc.six ? PATH_SPLIT6 : PATH_SPLIT)) tile_kib += tp.qfrag_kib;
      }
    }
  }
  if (npairs > 1 || tile_kib > kFusedTileKiB) fused = false;
  if (fused && rowres::comp_carve(dpmax, lds_stride(p.dim, 0)).total <= kMaxLdsBytes) {
    // evaluation order: components without pair terms first
    std::vector<int> order;
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < nc; ++i)
        if ((cd.comps[i].tiled[PATH_SPLIT].tp.any_pairwise != 0) == (pass == 1)) order.push_back(i);
    for (int mode = 0; mode < 3; ++mode) {
      std::vector<rowres::CompDesc> desc(cd.comps.size());
      for (size_t k = 0; k < order.size(); ++k) {
        const auto &cc = cd.comps[order[k]];
        const bool six = mode == 0 ? cc.six : mode == 2;
        const TiledProb &tp = cc.tiled[six ? PATH_SPLIT6 : PATH_SPLIT].tp;
        desc[k].tp = tp;
        desc[k].six = six ? 1 : 0;
        desc[k].unrotated = tp.rowwise;
        desc[k].index = order[k];
      }
      void *d = nullptr;
      if ((e = hipMalloc(&d, desc.size() * sizeof(rowres::CompDesc))) != hipSuccess) return e;
      cd.allocs.push_back(d);
      if ((e = hipMemcpy(d, desc.data(), desc.size() * sizeof(rowres::CompDesc), hipMemcpyHostToDevice)) != hipSuccess)
        return e;
      cd.rr_desc[mode] = d;
    }
    cd.rr_ok = true;
    cd.rr_dpmax = dpmax;
    cd.rr_S = lds_stride(p.dim, 0);
  }
  cd.ready = true;
  return hipSuccess;
}

void composite_scratch_needs(const CompositeDev &cd, int rows, size_t &pb, size_t &zb, size_t &gb, size_t &kb) {
  pb = zb = gb = kb = 0;
  auto acc_tiled = [&](const TiledDev (&t)[PATH_COUNT]) {
    for (int path = 0; path < PATH_COUNT; ++path)
      if (t[path].ready) {
        pb = std::max(pb, tiled_partials_bytes(t[path].tp, path, rows));
        zb = std::max(zb, tiled_z_bytes(t[path].tp, path, rows));
        kb = std::max(kb, tiled_pack_bytes(t[path].tp, path, rows));
      }
  };
  if (!cd.ready) return;
  if (!cd.is_composition) {
    acc_tiled(cd.tiled);
    return;
  }
  for (const auto &c : cd.comps)
    if (!c.resident) acc_tiled(c.tiled);
  gb = static_cast<size_t>(cd.comps.size()) * rows * sizeof(double);
}

bool carve_scratch(const CompositeDev &cd, void *base, size_t bytes, CompositeScratch &sc) {
  auto up256 = [](size_t v) { return (v + 255) & ~static_cast<size_t>(255); };
  for (int rows = kChunkRows; rows >= kTileRows; rows -= kTileRows) {
    size_t pb, zb, gb, kb;
    composite_scratch_needs(cd, rows, pb, zb, gb, kb);
    if (up256(pb) + up256(zb) + up256(gb) + up256(kb) > bytes) continue;
    unsigned char *p = static_cast<unsigned char *>(base);
    sc = CompositeScratch{};
    sc.cap = rows;
    sc.partials = p;
    sc.partials_bytes = pb;
    p += up256(pb);
    sc.zbuf = p;
    sc.zbuf_bytes = zb;
    p += up256(zb);
    sc.gbuf = p;
    sc.gbuf_bytes = gb;
    p += up256(gb);
    sc.pack = p;
    sc.pack_bytes = kb;
    return true;
  }
  return false;
}

hipError_t launch_composite(int path, bool split_auto, const CompositeDev &cd, const void *x, void *out, int n,
                            int num_cu, CompositeScratch &sc, hipStream_t st) {
  if (!cd.ready) return hipErrorNotSupported;
  const size_t esz = path == PATH_F64 ? 8 : 4;
  // basic functions and hybrids the row-resident kernel takes: one launch over all rows, no
  // scratch
  if (!cd.is_composition && rowres_fits(cd.tiled[path].tp, path))
    return launch_rowres(path, cd.kind_hint, cd.tiled[path].tp, x, out, n, num_cu, st);
  // compositions with every component on the row-resident kernel: one fused launch
  if (cd.is_composition && cd.rr_ok && is_split(path)) {
    const int mode = split_auto ? 0 : (path == PATH_SPLIT6 ? 2 : 1);
    return launch_rowres_comp(cd.rr_desc[mode], static_cast<int>(cd.comps.size()), cd.rr_dpmax, cd.rr_S,
                              static_cast<const float *>(x), n, cd.dim, cd.o64, cd.sig, cd.lam, cd.cb, cd.fopt,
                              static_cast<float *>(out), num_cu, st);
  }
  const int cap = sc.cap;
  if (cap < kTileRows || cap % kTileRows != 0) return hipErrorInvalidValue;
  for (int c0 = 0; c0 < n; c0 += cap) {
    const int ch = std::min(cap, n - c0);
    const unsigned char *xc = static_cast<const unsigned char *>(x) + static_cast<size_t>(c0) * cd.dim * esz;
    unsigned char *oc = static_cast<unsigned char *>(out) + static_cast<size_t>(c0) * esz;
    hipError_t e;
    if (!cd.is_composition) {
      e = launch_tiled(path, cd.kind_hint, cd.tiled[path].tp, xc, oc, ch, cap, sc.partials, sc.zbuf, sc.pack, st);
      if (e != hipSuccess) return e;
      continue;
    }
    const int nc = static_cast<int>(cd.comps.size());
    for (int i = 0; i < nc; ++i) {
      const CompositeDev::Component &cc = cd.comps[i];
      int cp = path;
      if (split_auto && is_split(path)) cp = cc.six ? PATH_SPLIT6 : PATH_SPLIT;
      unsigned char *gi = static_cast<unsigned char *>(sc.gbuf) + static_cast<size_t>(i) * cap * esz;
      if (cc.resident) {
        const DevProb &pb = cc.res[cp].pb;
        e = launch_resident(cp, pb, xc, gi, ch, resident_shape(cp, pb, ch, num_cu), st);
      } else {
        const TiledProb &ctp = cc.tiled[cp].tp;
        const int hint = ctp.nsegs == 1 && !cc.hybrid ? ctp.segs[0].kind : -1;
        if (rowres_fits(ctp, cp)) e = launch_rowres(cp, hint, ctp, xc, gi, ch, num_cu, st);
        else e = launch_tiled(cp, hint, ctp, xc, gi, ch, cap, sc.partials, sc.zbuf, sc.pack, st);
      }
      if (e != hipSuccess) return e;
    }
    e = launch_blend(path == PATH_F64, xc, ch, cd.dim, nc, cd.o64, cd.sig, cd.lam, cd.cb, sc.gbuf, cap, cd.fopt, oc,
                     st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace curob
