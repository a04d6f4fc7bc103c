// batch.cpp -- host side of the batched populations: problem tables, the work schedule, the
// captured HIP graph and the launch-shape autotuner.
#include "batch.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <queue>
#include <string>
#include <vector>

#include "../../include/curob.h"
#include "kernels.h"
#include "tables.h"

namespace curob {
int context_num_cu();
hipStream_t context_stream();
bool context_ready();
int set_error(int code, const std::string &msg);
}  // namespace curob

using namespace curob;

struct curob_batch {
  int k = 0;
  std::vector<int> fids, dims, counts, variants;
  std::vector<DevTables> tabs;     // one path per population
  std::vector<DevProb> host_probs; // device pointers inside
  std::vector<double> group_cost;  // estimated cost of one row group, per population
  std::vector<double> setup_cost;  // estimated cost of loading the tables, per population
  std::vector<void *> allocs;
  DevProb *d_probs = nullptr;
  int *d_variants = nullptr, *d_counts = nullptr;
  const void **d_xs = nullptr;
  void **d_outs = nullptr;
  int4 *d_items = nullptr;
  int *d_wg = nullptr;
  size_t items_cap = 0, wg_cap = 0;
  // launch shape
  int waves = 2, groups_per_item = 2, grid = 0, lds = 0, nitems = 0;
  bool bound = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;

  ~curob_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (auto &t : tabs) t.release();
    for (void *p : allocs) (void)hipFree(p);
  }
};

namespace {

int batch_fail(int code, const std::string &msg) { return set_error(code, msg); }

template <typename T>
hipError_t dev_alloc(curob_batch *b, T **p, size_t count) {
  void *d = nullptr;
  hipError_t e = hipMalloc(&d, std::max<size_t>(count, 1) * sizeof(T));
  if (e == hipSuccess) {
    b->allocs.push_back(d);
    *p = static_cast<T *>(d);
  }
  return e;
}

int lds_for(const curob_batch *b, int waves) {
  int lds = 0;
  for (int i = 0; i < b->k; ++i) {
    const int path = batch_variant(b->variants[i]).six ? PATH_SPLIT6 : PATH_SPLIT;
    lds = std::max(lds, lds_layout(path, b->host_probs[i], waves).total);
  }
  return lds;
}

// Items of up to gpi row groups, assigned longest first to the least loaded of `grid`
// workgroups; each workgroup's list is then ordered by population so that consecutive items
// share the LDS tables.
hipError_t plan(curob_batch *b, int waves, int gpi, int grid) {
  struct Item {
    int pop, g0, g1;
    double cost;
  };
  std::vector<Item> items;
  for (int i = 0; i < b->k; ++i) {
    const int ng = (b->counts[i] + kBatchRows - 1) / kBatchRows;
    for (int g0 = 0; g0 < ng; g0 += gpi) {
      const int g1 = std::min(ng, g0 + gpi);
      // the item's waves run its groups in ceil((g1 - g0) / waves) rounds
      const double rounds = std::ceil(static_cast<double>(g1 - g0) / waves);
      items.push_back(Item{i, g0, g1, rounds * b->group_cost[i] + b->setup_cost[i]});
    }
  }
  b->nitems = static_cast<int>(items.size());
  grid = std::max(1, std::min(grid, std::max(1, b->nitems)));
  std::stable_sort(items.begin(), items.end(), [](const Item &a, const Item &c) { return a.cost > c.cost; });
  std::vector<std::vector<Item>> per(grid);
  using Load = std::pair<double, int>;
  std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
  for (int w = 0; w < grid; ++w) heap.push({0.0, w});
  for (const Item &it : items) {
    Load l = heap.top();
    heap.pop();
    per[l.second].push_back(it);
    l.first += it.cost;
    heap.push(l);
  }
  std::vector<int4> flat;
  std::vector<int> wg(grid + 1, 0);
  for (int w = 0; w < grid; ++w) {
    std::sort(per[w].begin(), per[w].end(),
              [](const Item &a, const Item &c) { return a.pop != c.pop ? a.pop < c.pop : a.g0 < c.g0; });
    wg[w] = static_cast<int>(flat.size());
    for (const Item &it : per[w]) flat.push_back(make_int4(it.pop, it.g0, it.g1, 0));
  }
  wg[grid] = static_cast<int>(flat.size());
  hipError_t e = hipSuccess;
  if (flat.size() > b->items_cap) {
    if (b->d_items) {
      b->allocs.erase(std::find(b->allocs.begin(), b->allocs.end(), static_cast<void *>(b->d_items)));
      (void)hipFree(b->d_items);
      b->d_items = nullptr;
    }
    if ((e = dev_alloc(b, &b->d_items, flat.size())) != hipSuccess) return e;
    b->items_cap = flat.size();
  }
  if (wg.size() > b->wg_cap) {
    if (b->d_wg) {
      b->allocs.erase(std::find(b->allocs.begin(), b->allocs.end(), static_cast<void *>(b->d_wg)));
      (void)hipFree(b->d_wg);
      b->d_wg = nullptr;
    }
    if ((e = dev_alloc(b, &b->d_wg, wg.size())) != hipSuccess) return e;
    b->wg_cap = wg.size();
  }
  if (!flat.empty() && (e = hipMemcpy(b->d_items, flat.data(), flat.size() * sizeof(int4), hipMemcpyHostToDevice)) !=
                           hipSuccess)
    return e;
  if ((e = hipMemcpy(b->d_wg, wg.data(), wg.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess) return e;
  b->waves = waves;
  b->groups_per_item = gpi;
  b->grid = grid;
  b->lds = lds_for(b, waves);
  return hipSuccess;
}

hipError_t launch(const curob_batch *b, hipStream_t st) {
  if (b->nitems == 0) return hipSuccess;
  return launch_batch(b->d_probs, b->d_variants, b->d_xs, b->d_outs, b->d_counts, b->d_items, b->d_wg, b->grid, b->waves,
                      b->lds, st);
}

// Captures the current launch into a graph (on a stream of its own, default priority).
hipError_t capture(curob_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  hipStream_t s = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t le = launch(b, s);
    e = hipStreamEndCapture(s, &b->graph);
    if (le != hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(s);
  return e;
}

bool shape_ok(const curob_batch *b, int waves, int gpi, int grid) {
  return waves >= 1 && waves <= kBatchMaxWaves && gpi >= 1 && grid >= 1 && lds_for(b, waves) <= kMaxLdsBytes;
}

}  // namespace

extern "C" {

int curob_batch_create(int k, const int *fids, const int *dims, const int *counts, unsigned long long seed,
                       curob_batch **out) {
  if (out) *out = nullptr;
  if (!context_ready()) return batch_fail(CUROB_E_STATE, "library is not initialised (call initialize first)");
  if (!out || !fids || !dims || !counts) return batch_fail(CUROB_E_ARG, "null pointer");
  if (k < 1 || k > 65536) return batch_fail(CUROB_E_ARG, "k must be in 1..65536");
  for (int i = 0; i < k; ++i) {
    if (fids[i] < 0 || fids[i] > 22) return batch_fail(CUROB_E_FID, "batch functions must be Tab. 1 ids 0..22");
    if (dims[i] < 2 || dims[i] > 16 * kMaxMT) return batch_fail(CUROB_E_ARG, "batch dimensions must be in 2..128");
    if (dims[i] < min_dimension(fids[i])) return batch_fail(CUROB_E_ARG, "dimension below the formula's minimum");
    if (counts[i] < 0) return batch_fail(CUROB_E_ARG, "counts must be >= 0");
  }
  auto *b = new curob_batch();
  b->k = k;
  b->fids.assign(fids, fids + k);
  b->dims.assign(dims, dims + k);
  b->counts.assign(counts, counts + k);
  b->variants.resize(k);
  for (int i = 0; i < k; ++i) b->variants[i] = batch_variant_of(fids[i], dims[i]);
  b->tabs.resize(k);
  b->host_probs.resize(k);
  b->group_cost.resize(k);
  b->setup_cost.resize(k);
  hipError_t e = hipSuccess;
  for (int i = 0; i < k; ++i) {
    const FnSpec &t = fn_spec(fids[i]);
    const BatchVariant v = batch_variant(b->variants[i]);
    const int path = v.six ? PATH_SPLIT6 : PATH_SPLIT;
    Problem p = make_basic(fids[i], dims[i], seed, (kBatchKeyBase + static_cast<uint32_t>(i)) << 8, t.s, t.c,
                           t.rotated, false);
    HostTables ht;
    std::string err;
    if (!build_host_tables(p, path, ht, err)) {
      delete b;
      return batch_fail(CUROB_E_ARG, err);
    }
    if (ht.pb.kind != v.kind || ht.pb.rotated != v.rot || needs_six_products(fids[i], dims[i]) != (v.six != 0)) {
      delete b;
      return batch_fail(CUROB_E_ARG, "batch variant table disagrees with the problem tables");
    }
    if ((e = upload_tables(ht, b->tabs[i])) != hipSuccess) break;
    b->host_probs[i] = b->tabs[i].pb;
    const DevProb &pb = b->host_probs[i];
    // row-group cost: staging the rows plus the rotation's MFMA tiles (x3 or x6 products)
    b->group_cost[i] = 2.0 * pb.D + (pb.rotated ? pb.ntiles * (v.six ? 12.0 : 6.0) : 0.0) + 16.0 * pb.MT;
    b->setup_cost[i] = lds_layout(path, pb, 1).fixed / 256.0;
  }
  if (e == hipSuccess) e = dev_alloc(b, &b->d_probs, k);
  if (e == hipSuccess) e = dev_alloc(b, &b->d_variants, k);
  if (e == hipSuccess) e = dev_alloc(b, &b->d_counts, k);
  if (e == hipSuccess) e = dev_alloc(b, &b->d_xs, k);
  if (e == hipSuccess) e = dev_alloc(b, &b->d_outs, k);
  if (e == hipSuccess) e = hipMemcpy(b->d_probs, b->host_probs.data(), k * sizeof(DevProb), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_variants, b->variants.data(), k * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_counts, counts, k * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(b->d_xs, 0, k * sizeof(void *));
  if (e == hipSuccess) e = hipMemset(b->d_outs, 0, k * sizeof(void *));
  // default shape until tuned: two waves, two row groups per item, two workgroups per CU
  if (e == hipSuccess) e = plan(b, 2, 2, 2 * context_num_cu());
  if (e == hipSuccess && b->lds > kMaxLdsBytes) e = plan(b, 1, 2, 2 * context_num_cu());
  if (e != hipSuccess) {
    delete b;
    return batch_fail(CUROB_E_HIP, std::string("creating the batch: ") + hipGetErrorString(e));
  }
  *out = b;
  return CUROB_OK;
}

int curob_batch_bind(curob_batch *b, const float *const *d_xs, float *const *d_outs) {
  if (!b || !d_xs || !d_outs) return batch_fail(CUROB_E_ARG, "null pointer");
  for (int i = 0; i < b->k; ++i)
    if (b->counts[i] > 0 && (!d_xs[i] || !d_outs[i]))
      return batch_fail(CUROB_E_ARG, "null buffer for a population with rows");
  // the previous replay may still read the pointer tables
  hipError_t e = hipStreamSynchronize(context_stream());
  if (e == hipSuccess) e = hipMemcpy(b->d_xs, d_xs, b->k * sizeof(void *), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_outs, d_outs, b->k * sizeof(void *), hipMemcpyHostToDevice);
  if (e == hipSuccess && !b->exec) e = capture(b);
  if (e != hipSuccess) return batch_fail(CUROB_E_HIP, std::string("binding the batch: ") + hipGetErrorString(e));
  b->bound = true;
  return CUROB_OK;
}

int curob_batch_run(curob_batch *b) {
  if (!b) return batch_fail(CUROB_E_ARG, "null batch");
  if (!b->bound) return batch_fail(CUROB_E_STATE, "bind the batch's buffers first");
  if (b->nitems == 0) return CUROB_OK;
  hipError_t e = hipGraphLaunch(b->exec, context_stream());
  if (e != hipSuccess) return batch_fail(CUROB_E_HIP, std::string("graph launch: ") + hipGetErrorString(e));
  return CUROB_OK;
}

int curob_batch_run_direct(curob_batch *b) {
  if (!b) return batch_fail(CUROB_E_ARG, "null batch");
  if (!b->bound) return batch_fail(CUROB_E_STATE, "bind the batch's buffers first");
  hipError_t e = launch(b, context_stream());
  if (e != hipSuccess) return batch_fail(CUROB_E_HIP, std::string("batch launch: ") + hipGetErrorString(e));
  return CUROB_OK;
}

int curob_batch_configure(curob_batch *b, int waves, int groups_per_item, int grid) {
  if (!b) return batch_fail(CUROB_E_ARG, "null batch");
  if (!shape_ok(b, waves, groups_per_item, grid))
    return batch_fail(CUROB_E_ARG, "waves must be 1..4 (LDS permitting), groups_per_item and grid >= 1");
  hipError_t e = hipStreamSynchronize(context_stream());
  if (e == hipSuccess) e = plan(b, waves, groups_per_item, grid);
  if (e == hipSuccess && b->bound) e = capture(b);
  if (e != hipSuccess) return batch_fail(CUROB_E_HIP, std::string("configuring the batch: ") + hipGetErrorString(e));
  return CUROB_OK;
}

int curob_batch_shape(const curob_batch *b, int *waves, int *groups_per_item, int *grid, int *nitems) {
  if (!b) return batch_fail(CUROB_E_ARG, "null batch");
  if (waves) *waves = b->waves;
  if (groups_per_item) *groups_per_item = b->groups_per_item;
  if (grid) *grid = b->grid;
  if (nitems) *nitems = b->nitems;
  return CUROB_OK;
}

int curob_batch_tune(curob_batch *b, int reps, float *best_us) {
  if (!b) return batch_fail(CUROB_E_ARG, "null batch");
  if (!b->bound) return batch_fail(CUROB_E_STATE, "bind the batch's buffers before tuning (it times real launches)");
  if (reps < 1) reps = 1;
  hipStream_t st = context_stream();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const int cu = context_num_cu();
  float best = 1e30f;
  int bw = b->waves, bg = b->groups_per_item, bgrid = b->grid;
  const int waves_c[] = {1, 2, 4};
  const int gpi_c[] = {1, 2, 4, 8};
  const int grid_c[] = {cu / 2, cu, 2 * cu, 4 * cu};
  for (int w : waves_c) {
    for (int gm : gpi_c) {
      for (int gr : grid_c) {
        if (e != hipSuccess) break;
        const int gpi = w * gm;
        if (!shape_ok(b, w, gpi, gr)) continue;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) break;
        if ((e = plan(b, w, gpi, gr)) != hipSuccess) break;
        if (b->grid < gr && gr != grid_c[0]) continue;  // fewer items than workgroups: same as a smaller grid
        for (int r = 0; r < 2 && e == hipSuccess; ++r) e = launch(b, st);
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch(b, st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        const float us = 1000.0f * ms / reps;
        if (e == hipSuccess && us < best) {
          best = us;
          bw = w;
          bg = gpi;
          bgrid = b->grid;
        }
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e == hipSuccess) e = plan(b, bw, bg, bgrid);
  if (e == hipSuccess) e = capture(b);
  if (e != hipSuccess) return batch_fail(CUROB_E_HIP, std::string("tuning the batch: ") + hipGetErrorString(e));
  if (best_us) *best_us = best;
  return CUROB_OK;
}

int curob_batch_destroy(curob_batch *b) {
  if (!b) return CUROB_OK;
  (void)hipStreamSynchronize(context_stream());
  delete b;
  return CUROB_OK;
}

}  // extern "C"
