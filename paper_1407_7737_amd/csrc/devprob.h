// devprob.h -- the per-problem device tables handed to the evaluation kernels by value.
// Shared by the host table builder and the kernels; plain data only.
#pragma once

#include <cstdint>

namespace curob {

// Arithmetic of one evaluation path.
enum Path : int {
  PATH_SPLIT = 0,   // FP32 data, rotation as three BF16 MFMA products (hi*hi + hi*lo + lo*hi)
  PATH_F32 = 1,     // FP32 data, rotation on FP32 MFMA
  PATH_F64 = 2,     // FP64 data, rotation on FP64 MFMA
  PATH_SPLIT6 = 3,  // FP32 data, three-term BF16 splits of y and Q, six MFMA products
  PATH_COUNT = 4
};

inline constexpr bool is_split(int path) { return path == PATH_SPLIT || path == PATH_SPLIT6; }
// bf16 fragments stored per rotation tile: hi, lo (x3) or hi, mid, lo (x6)
inline constexpr int split_terms(int path) { return path == PATH_SPLIT6 ? 3 : 2; }

// Tile geometry of the block-diagonal rotation in packed (group-ordered) variable space.
// The MFMA computes Z^T = Qp Y^T tile by tile: Qp is the packed block-diagonal matrix,
// m-tiles are 16 output positions, k-tiles are KW input positions (32 for BF16, 4 for FP32/64).
constexpr int kMaxMT = 8;          // m-tiles supported by the resident kernel (dimension <= 128)
constexpr int kRowsPerBlock = 16;  // population rows per MFMA column block (the MFMA N dimension)

inline constexpr int kw_of(int path) { return is_split(path) ? 32 : 4; }
// 16-row column blocks a wave evaluates per iteration.  One on every path: two would let each
// rotation tile read from LDS feed two MFMAs, but would double the registers and the LDS slice
// of a wave and halve the waves a CU holds, and the kernel needs the waves to hide latency.
inline constexpr int blocks_of(int) { return 1; }

struct DevProb {
  // The per-problem tables, laid out exactly as the fixed part of the kernel's LDS carve
  // (kernels.h lds_layout), in one device block the kernel copies with a single pass:
  //   rotation tiles: nonzero tiles of s*Qp in MFMA operand order (path-specific layout);
  //   gather offsets: packed position -> byte offset of its variable in an LDS row (KT*KW
  //     entries, padding -> the zero slot at D);
  //   o_hi: the shift rounded to the path's type, original variable order (D entries), or on
  //     the split paths packed order (max(KT*KW, 16*MT) entries, zeros past D);
  //   c': per packed position (16*MT entries), c minus the rotated, scaled rounding error of the
  //     shift on the FP32 paths;
  //   coefficients per packed position (elliptic weights, 1/sqrt(i), ...);
  //   successors: per packed position the packed position of the formula successor or -1;
  //   k ranges: per m-tile first k-tile, last k-tile, first tile index and, on the split paths,
  //     4 * first k-tile + (last - first).
  const void *image;  // device memory owned by the library
  int image_bytes;    // the fixed part of the LDS carve, a multiple of 16
  int D;                 // dimension
  int S;                 // LDS row stride in elements (4*odd, >= D+1, and >= 16*MT unless the rows
                         // are loaded directly, kernels.h direct_rows)
  int KT;                // k-tiles
  int MT;                // m-tiles
  int ntiles;            // nonzero tiles
  int rotated;           // 0: z = s*y + c' directly
  int kind;              // formula family (problem.h Kind)
  int Df;                // dimension seen by the formula
  double bias;           // f_opt
  double kparam;         // family parameter (Katsuura exponent 10/D^1.2)
  double scale;          // s, applied in the formula phase when the problem is unrotated
  double padc[3];        // what the 16*MT - D padded positions add to each sum, removed at the end
};

}  // namespace curob
