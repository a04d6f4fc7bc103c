// tiled.h -- the tiled evaluation path: basic functions above the resident kernel's dimension
// range and every hybrid function (Sec. 5).  Device tables, host builder, launchers.
//
// The packed variable space is cut into rotation blocks (the three groups of Sec. 1.2, or the
// hybrid groups of Sec. 5), each padded to a multiple of 32 positions so that no MFMA tile
// straddles two blocks.  A workgroup computes one tile of 64 population rows x up to 64 outputs
// of one block, applies the formula and leaves compensated per-row partial sums in a scratch
// buffer; a second kernel combines the partials of each formula segment per row.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "devprob.h"
#include "problem.h"

namespace curob {

constexpr int kRowTiles = 8;                    // 16-row MFMA column blocks per workgroup tile
constexpr int kTileRows = 16 * kRowTiles;       // population rows per workgroup tile
constexpr int kTileK = 32;         // packed positions staged per k step
constexpr int kGroupMTiles = 8;    // m-tiles (of 16 outputs) per workgroup output group
constexpr int kPartialSlots = 8;   // per (row, output group): s0 c0 s1 c1 s2 c2 product pad
constexpr int kMaxSegments = 16;   // formula segments per tiled problem
constexpr int kChunkRows = 65536;  // rows per pass (bounds the scratch buffers)
constexpr int kPackLdsBytes = 150 * 1024;  // LDS budget of a pack workgroup
constexpr int kNumXcd = 8;                 // accelerator complex dies the workgroups are dealt to

struct TiledSeg {
  int kind;      // formula family of the segment
  int base;      // Tab. 1 id
  int g0, g1;    // output groups [g0, g1) of this segment
  int p0, p1;    // padded positions [p0, p1)
  int n;         // dimension the formula sees
  int pairwise;  // 1: terms need z of the successor
  double kparam; // family parameter (Katsuura exponent)
  double padc[3];
};

// One output group: m-tiles [m0, m0 + count) of a block.
struct TiledGroup {
  int block, m0, count, seg;
};

struct TiledProb {
  // device pointers
  const int *gidx;      // padded position -> original variable, -1 for padding (Dp entries)
  const void *oh;       // shift rounded to the path's type (D entries)
  const void *cz;       // c' per padded position
  const void *coef;     // coefficient per padded position
  const int *succ;      // successor padded position (pairwise) or -1
  const void *qfrag;    // dense tiles of s*Q per block, MFMA A-operand order
  const int4 *blocks;   // per block: padded offset, padded size, first tile, k-tiles
  const int4 *groups;   // per output group: block, first m-tile, m-tile count, segment
  // row-resident kernel (split paths): per padded position the byte offset of its variable in
  // an LDS row (padding: the zero slot at column D) and o_hi in packed order (0 for padding)
  const uint16_t *goff;
  const float *ohp;
  int S;          // LDS row stride (floats) of the row-resident kernel
  int D, Dp, nblocks, ngroups, nsegs;
  int any_pairwise;
  int pair_mtiles_max;  // m-tiles of the largest rotation block with pair terms (host use)
  int mtiles_max;       // m-tiles of the largest rotation block (host use)
  int qfrag_kib;        // size of the rotation tiles in KiB (host use)
  int rowwise;    // unrotated basic problem: z = s (x - o) + c' per variable, no MFMA work
  double scale0;  // s of that problem
  double bias;
  TiledSeg segs[kMaxSegments];
};

struct TiledDev {
  std::vector<void *> allocs;
  TiledProb tp{};
  bool ready = false;
  void release();
};

// Builds and uploads the tiled tables of a basic or hybrid problem for one path.
hipError_t build_tiled(const Problem &p, int path, TiledDev &td, std::string &err);

// Scratch the tiled kernels need for a chunk of `rows` rows: partial sums, (pairwise) z and the
// packed B operands (bytes per packed position and row: 2 per bf16 term, 4 FP32, 8 FP64).
size_t tiled_partials_bytes(const TiledProb &tp, int path, int rows);
size_t tiled_z_bytes(const TiledProb &tp, int path, int rows);
size_t tiled_pack_bytes(const TiledProb &tp, int path, int rows);

// Whether the row-resident kernel takes this problem on this path (split paths, rotated, the
// rows and tables fit the LDS); it needs no scratch.
bool rowres_fits(const TiledProb &tp, int path);
// Evaluates rows [0, n) of x into out with the row-resident kernel (any n).
hipError_t launch_rowres(int path, int kind_hint, const TiledProb &tp, const void *x, void *out, int n, int num_cu,
                         hipStream_t st);

// Evaluates rows [0, n) of x into out using scratch buffers sized for cap rows (n <= cap, cap a
// multiple of kTileRows).
hipError_t launch_tiled(int path, int kind_hint, const TiledProb &tp, const void *x, void *out, int n, int cap,
                        void *partials, void *zbuf, void *pack, hipStream_t st);

}  // namespace curob
