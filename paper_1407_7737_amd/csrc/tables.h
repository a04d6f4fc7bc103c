// tables.h -- host construction of the device tables for one problem and one path.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "devprob.h"
#include "problem.h"

namespace curob {

// Device memory owned by one problem for one path.
struct DevTables {
  std::vector<void *> allocs;
  DevProb pb{};
  bool ready = false;
  void release();
};

// Host-side images of the tables (exposed for CPU checks of the layout).
struct HostTables {
  int path = 0;
  std::vector<unsigned char> oh, cz, coef, qfrag;
  std::vector<uint16_t> goff;
  std::vector<int16_t> succ;
  std::vector<int> mtab;
  DevProb pb{};
};

// Builds the images for a basic problem of dimension <= 128 (the resident kernel's range).
// Returns false with a message when the problem is outside that range.
bool build_host_tables(const Problem &p, int path, HostTables &ht, std::string &err);

// Uploads the images; pb pointers then refer to device memory.
hipError_t upload_tables(const HostTables &ht, DevTables &dt);

// Round-to-nearest-even float -> bf16 bits, as the device conversion does.
uint16_t bf16_bits_rne(float f);
float bf16_bits_to_float(uint16_t h);

// LDS row stride: the smallest 4u >= max(D + 1, m) with u odd (16 rows then fall in distinct
// banks), m the padded position count.
int lds_stride(int D, int m);

// What one padded Schwefel position (z = 0, the optimum of g1) adds to the row sum of terms
// 418.9829 - g1: on the FP32 paths the series value at 0, on the FP64 path the term itself.
double schwefel_pad_term(bool f64);

}  // namespace curob
