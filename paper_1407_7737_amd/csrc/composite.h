// composite.h -- everything the resident kernel does not cover: basic functions above its
// dimension range and hybrids (the tiled path), and compositions (Sec. 6), whose components are
// evaluated by the resident or tiled path and blended with FP64 weights.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "problem.h"
#include "tables.h"
#include "tiled.h"

namespace curob {

struct CompositeDev {
  struct Component {
    TiledDev tiled[PATH_COUNT];
    DevTables res[PATH_COUNT];
    bool resident = false;
    bool six = false;  // split mode: six products
    bool hybrid = false;
  };
  bool ready = false;
  bool is_composition = false;
  int dim = 0;
  TiledDev tiled[PATH_COUNT];  // basic (large dimension) or hybrid
  int kind_hint = -1;          // formula family for a basic problem, -1 for hybrids
  std::vector<Component> comps;
  std::vector<void *> allocs;  // blend tables
  const double *o64 = nullptr; // component optima, ncomp x dim
  const double *sig = nullptr, *lam = nullptr, *cb = nullptr;
  double fopt = 100.0;
  // fused composition on the split paths (every component on the same staged rows): component
  // descriptors per split mode (0: three or six products per component, 1: three, 2: six)
  bool rr_ok = false;
  const void *rr_desc[3] = {nullptr, nullptr, nullptr};
  int rr_dpmax = 0, rr_S = 0;
  void release();
};

// Scratch shared by all composite evaluations of a context: buffers for a chunk of `cap` rows
// (rows are evaluated in passes of cap).  reserve/release manage library-allocated buffers;
// carve_scratch points the four buffers into caller-provided memory instead.
struct CompositeScratch {
  void *partials = nullptr;
  void *zbuf = nullptr;
  void *gbuf = nullptr;
  void *pack = nullptr;
  size_t partials_bytes = 0, zbuf_bytes = 0, gbuf_bytes = 0, pack_bytes = 0;
  int cap = kChunkRows;
  hipError_t reserve(size_t pb, size_t zb, size_t gb, size_t kb);
  void release();
};

// Uploads whatever the composite kernels need for p.  Basic problems within the resident
// kernel's range need nothing here.
hipError_t build_composite(const Problem &p, CompositeDev &cd, std::string &err);

// Scratch sizes the problem needs for chunks of `rows` rows.
void composite_scratch_needs(const CompositeDev &cd, int rows, size_t &pb, size_t &zb, size_t &gb, size_t &kb);

// Points sc into the `bytes` of device memory at base (256-byte aligned), with the largest chunk
// of rows (a multiple of kTileRows, at most kChunkRows) whose buffers fit.  Returns false when
// not even kTileRows rows fit.  Nothing is allocated.
bool carve_scratch(const CompositeDev &cd, void *base, size_t bytes, CompositeScratch &sc);

// Evaluates n rows of x into out.  path is the arithmetic of the call; in split mode
// (split_auto) the components of a composition pick three or six products per formula.
hipError_t launch_composite(int path, bool split_auto, const CompositeDev &cd, const void *x, void *out, int n,
                            int num_cu, CompositeScratch &sc, hipStream_t st);

}  // namespace curob
