// api.cpp -- the C ABI of include/curob.h: state machine, validation, problem registry,
// dispatch to the evaluation kernels and the host-pointer wrappers (Sec. 1.3).
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>

#include "../../include/curob.h"
#include "batch.h"
#include "composite.h"
#include "kernels.h"
#include "problem.h"
#include "tables.h"

// Device memory of the allocation-free entry point func_evaluatef_noalloc: the tiled and
// composition kernels' scratch (partial sums, pairwise z, packed operands, component values)
// carved out of one file-scope array per device.  Host code never uses this name as an address:
// it takes the device address from hipGetSymbolAddress once per device and passes that on.
constexpr size_t kNoallocScratchBytes = CUROB_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace curob {

hipError_t launch_de_trial(bool f64, const void *pop, void *trial, int np, int D, double F, double CR, uint64_t seed,
                           const unsigned long long *gen, hipStream_t st);
hipError_t launch_de_select(bool f64, void *pop, void *fit, const void *trial, const void *ftrial, int np, int D,
                            unsigned long long *gen, hipStream_t st);

namespace {

struct Entry {
  Problem host;
  DevTables dev[PATH_COUNT];
  CompositeDev comp;  // hybrids and compositions
  ~Entry() {
    for (auto &d : dev) d.release();
    comp.release();
  }
};

struct Context {
  bool ready = false;
  int dim = 0;
  int maxc = 0;
  uint64_t seed = 0;
  int device = 0;
  int num_cu = 0;
  int mode = CUROB_MODE_SPLIT;
  hipStream_t stream = nullptr;
  std::map<int, std::unique_ptr<Entry>> entries;
  // Tab. 1 ids whose definition leaves them undefined at this dimension, with the reason
  std::map<int, std::string> undefined;
  CompositeScratch scratch;   // tiled partial sums, pairwise z, composition components
  void *stage_x = nullptr;    // maxc * dim doubles, for the h_ wrappers
  void *stage_out = nullptr;  // maxc doubles
  // The scratch is shared by every tiled and composition call: a call on another stream than
  // the previous scratch user first waits for this event, recorded after that call.
  hipEvent_t scratch_done = nullptr;
  hipStream_t scratch_stream = nullptr;
  bool scratch_used = false;
};

Context g_ctx;
std::string g_err;

// device -> address of that device's copy of `scratch` (looked up once per device)
std::map<int, void *> g_noalloc_scratch;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(CUROB_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

void free_context() {
  clear_shape_overrides();
  g_ctx.entries.clear();
  g_ctx.scratch.release();
  if (g_ctx.stage_x) (void)hipFree(g_ctx.stage_x);
  if (g_ctx.stage_out) (void)hipFree(g_ctx.stage_out);
  if (g_ctx.scratch_done) (void)hipEventDestroy(g_ctx.scratch_done);
  g_ctx = Context{};
}

// Builds device data for a problem on every path: basic problems within the resident kernel's
// dimension range get its tables, everything else the tiled / composition tables, and the
// context's scratch grows to what the problem needs.
int prepare_entry(Entry &e) {
  const Problem &p = e.host;
  if (p.type == Problem::BASIC) {
    for (int path = 0; path < PATH_COUNT; ++path) {
      if (p.dim <= 16 * kMaxMT) {
        HostTables ht;
        std::string err;
        if (!build_host_tables(p, path, ht, err)) return fail(CUROB_E_ARG, "%s", err.c_str());
        hipError_t he = upload_tables(ht, e.dev[path]);
        if (he != hipSuccess) return hip_fail(he, "uploading problem tables");
      }
    }
  }
  std::string err;
  hipError_t he = build_composite(p, e.comp, err);
  if (he != hipSuccess) {
    if (!err.empty()) return fail(CUROB_E_ARG, "%s", err.c_str());
    return hip_fail(he, "uploading composite tables");
  }
  size_t pb = 0, zb = 0, gb = 0, kb = 0;
  composite_scratch_needs(e.comp, kChunkRows, pb, zb, gb, kb);
  he = g_ctx.scratch.reserve(pb, zb, gb, kb);
  if (he != hipSuccess) return hip_fail(he, "allocating scratch");
  return CUROB_OK;
}

int register_problem(int id, Problem &&p) {
  auto e = std::make_unique<Entry>();
  e->host = std::move(p);
  int rc = prepare_entry(*e);
  if (rc != CUROB_OK) return rc;
  g_ctx.entries[id] = std::move(e);
  return CUROB_OK;
}

// FP32 entry point: the arithmetic path for a problem under the current mode.
int fp32_path(int fid) {
  switch (g_ctx.mode) {
    case CUROB_MODE_FP32: return PATH_F32;
    case CUROB_MODE_SPLIT_BF16X3: return PATH_SPLIT;
    case CUROB_MODE_SPLIT_BF16X6: return PATH_SPLIT6;
    default: break;
  }
  auto it = g_ctx.entries.find(fid);
  if (it == g_ctx.entries.end()) return PATH_SPLIT;
  const Problem &p = it->second->host;
  // compositions choose per component inside launch_composite
  if (p.type == Problem::COMPOSITION) return PATH_SPLIT;
  return problem_needs_six(p) ? PATH_SPLIT6 : PATH_SPLIT;
}

// An id without an entry: undefined at this dimension (with the reason), or never registered.
int not_defined(int fid) {
  auto u = g_ctx.undefined.find(fid);
  if (u != g_ctx.undefined.end())
    return fail(CUROB_E_FID, "function id %d is not defined for dim %d: %s", fid, g_ctx.dim, u->second.c_str());
  return fail(CUROB_E_FID, "function id %d is not defined for dim %d", fid, g_ctx.dim);
}

int check_ready() {
  if (!g_ctx.ready) return fail(CUROB_E_STATE, "library is not initialised (call initialize first)");
  return CUROB_OK;
}

int check_eval_args(int fid, const void *x, int n, const void *out, Entry **entry) {
  int rc = check_ready();
  if (rc != CUROB_OK) return rc;
  auto it = g_ctx.entries.find(fid);
  if (it == g_ctx.entries.end()) return not_defined(fid);
  if (n < 0) return fail(CUROB_E_ARG, "n must be >= 0 (got %d)", n);
  if (n > g_ctx.maxc) return fail(CUROB_E_CAPACITY, "n = %d exceeds max_concurrency %d", n, g_ctx.maxc);
  if (n > 0 && (x == nullptr || out == nullptr)) return fail(CUROB_E_ARG, "null pointer with n > 0");
  *entry = it->second.get();
  return CUROB_OK;
}

int evaluate(int path, int fid, const void *x, int n, void *out) {
  Entry *e = nullptr;
  int rc = check_eval_args(fid, x, n, out, &e);
  if (rc != CUROB_OK || n == 0) return rc;
  hipError_t he;
  if (e->host.type == Problem::BASIC && e->dev[path].ready) {
    const DevProb &pb = e->dev[path].pb;
    he = launch_resident(path, pb, x, out, n, resident_shape(path, pb, n, g_ctx.num_cu), g_ctx.stream);
  } else if (e->comp.ready) {
    const bool split_auto = g_ctx.mode == CUROB_MODE_SPLIT && path != PATH_F64;
    // order this call after the previous user of the shared scratch when that ran on another
    // stream; under stream capture the caller orders its captured work itself
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    he = hipStreamIsCapturing(g_ctx.stream, &cap);
    if (he != hipSuccess) return hip_fail(he, "querying stream capture");
    const bool track = cap == hipStreamCaptureStatusNone;
    if (track && g_ctx.scratch_used && g_ctx.scratch_stream != g_ctx.stream) {
      he = hipStreamWaitEvent(g_ctx.stream, g_ctx.scratch_done, 0);
      if (he != hipSuccess) return hip_fail(he, "ordering scratch use across streams");
    }
    he = launch_composite(path, split_auto, e->comp, x, out, n, g_ctx.num_cu, g_ctx.scratch, g_ctx.stream);
    if (he == hipSuccess && track) {
      he = hipEventRecord(g_ctx.scratch_done, g_ctx.stream);
      g_ctx.scratch_stream = g_ctx.stream;
      g_ctx.scratch_used = true;
    }
  } else {
    return fail(CUROB_E_HIP, "function id %d has no device tables", fid);
  }
  if (he != hipSuccess) return hip_fail(he, "kernel launch");
  return CUROB_OK;
}

template <typename T>
int h_evaluate(int path, int fid, const T *hx, int n, T *hout) {
  Entry *e = nullptr;
  int rc = check_eval_args(fid, hx, n, hout, &e);
  if (rc != CUROB_OK || n == 0) return rc;
  const size_t xb = static_cast<size_t>(n) * g_ctx.dim * sizeof(T);
  hipError_t he = hipMemcpyAsync(g_ctx.stage_x, hx, xb, hipMemcpyHostToDevice, g_ctx.stream);
  if (he != hipSuccess) return hip_fail(he, "copying inputs to the device");
  rc = evaluate(path, fid, g_ctx.stage_x, n, g_ctx.stage_out);
  if (rc != CUROB_OK) return rc;
  he = hipMemcpyAsync(hout, g_ctx.stage_out, static_cast<size_t>(n) * sizeof(T), hipMemcpyDeviceToHost, g_ctx.stream);
  if (he != hipSuccess) return hip_fail(he, "copying results to the host");
  he = hipStreamSynchronize(g_ctx.stream);
  if (he != hipSuccess) return hip_fail(he, "waiting for the evaluation");
  return CUROB_OK;
}

// The part of a problem an export call describes: the problem itself (comp < 0) or component
// comp of a composition.
int select_part(const Problem &top, int comp, const Problem **part) {
  if (comp < 0) {
    *part = &top;
    return CUROB_OK;
  }
  if (top.type != Problem::COMPOSITION) return fail(CUROB_E_ARG, "only compositions have components");
  if (comp >= static_cast<int>(top.comps.size()))
    return fail(CUROB_E_ARG, "component %d out of range (%d components)", comp, static_cast<int>(top.comps.size()));
  *part = &top.comps[static_cast<size_t>(comp)];
  return CUROB_OK;
}

int export_info(const Problem &top, int comp, int *type, int *count, int *nseg) {
  const Problem *p = nullptr;
  int rc = select_part(top, comp, &p);
  if (rc != CUROB_OK) return rc;
  if (type) *type = p->type;
  if (count) *count = p->type == Problem::COMPOSITION ? static_cast<int>(p->comps.size()) : static_cast<int>(p->Q.size());
  if (nseg) *nseg = static_cast<int>(p->segs.size());
  return CUROB_OK;
}

int export_structure(const Problem &top, int comp, double *o, int *perm, int *sizes, double *blocks, int *bases,
                     double *scale, double *offset) {
  const Problem *p = nullptr;
  int rc = select_part(top, comp, &p);
  if (rc != CUROB_OK) return rc;
  if (p->type == Problem::COMPOSITION)
    return fail(CUROB_E_ARG, "a composition has no single structure: name a component");
  if (o) std::memcpy(o, p->o.data(), sizeof(double) * p->o.size());
  if (perm) std::memcpy(perm, p->orig.data(), sizeof(int) * p->orig.size());
  size_t off = 0;
  for (size_t k = 0; k < p->Q.size(); ++k) {
    if (sizes) sizes[k] = p->blk_n[k];
    if (blocks) std::memcpy(blocks + off, p->Q[k].data(), sizeof(double) * p->Q[k].size());
    off += p->Q[k].size();
  }
  for (size_t i = 0; i < p->segs.size(); ++i) {
    if (bases) bases[i] = p->segs[i].base;
    if (scale) scale[i] = p->segs[i].s;
    if (offset) offset[i] = p->segs[i].c;
  }
  return CUROB_OK;
}

int export_composition(const Problem &p, double *sigma, double *lambda, double *bias) {
  if (p.type != Problem::COMPOSITION) return fail(CUROB_E_ARG, "not a composition");
  for (size_t i = 0; i < p.comps.size(); ++i) {
    if (sigma) sigma[i] = p.sigma[i];
    if (lambda) lambda[i] = p.lambda[i];
    if (bias) bias[i] = p.cbias[i];
  }
  return CUROB_OK;
}

int find_entry(int fid, const Problem **p) {
  int rc = check_ready();
  if (rc != CUROB_OK) return rc;
  auto it = g_ctx.entries.find(fid);
  if (it == g_ctx.entries.end()) return not_defined(fid);
  *p = &it->second->host;
  return CUROB_OK;
}

// A Tab. 1 problem generated on the host only (no device, no context).
int generate_tab1(int fid, int dim, unsigned long long seed, Problem &p) {
  if (fid < 0 || fid > 36) return fail(CUROB_E_FID, "fid must be in 0..36");
  if (dim < 2) return fail(CUROB_E_ARG, "dim must be >= 2");
  try {
    p = make_tab1(fid, dim, seed);
  } catch (const std::exception &ex) {
    return fail(CUROB_E_ARG, "%s", ex.what());
  }
  return CUROB_OK;
}

}  // namespace

int context_num_cu() { return g_ctx.num_cu; }
bool context_ready() { return g_ctx.ready; }
hipStream_t context_stream() { return g_ctx.stream; }
int set_error(int code, const std::string &msg) { return fail(code, "%s", msg.c_str()); }

}  // namespace curob

using namespace curob;

extern "C" {

int initialize(int dim, int max_concurrency, unsigned long long seed) {
  if (g_ctx.ready) return fail(CUROB_E_STATE, "already initialised (call dispose first)");
  if (dim < 2) return fail(CUROB_E_ARG, "dim must be >= 2 (got %d)", dim);
  if (max_concurrency < 1) return fail(CUROB_E_ARG, "max_concurrency must be >= 1 (got %d)", max_concurrency);
  int ndev = 0;
  hipError_t he = hipGetDeviceCount(&ndev);
  if (he != hipSuccess || ndev < 1) return fail(CUROB_E_HIP, "no HIP device available");
  he = hipGetDevice(&g_ctx.device);
  if (he != hipSuccess) return hip_fail(he, "hipGetDevice");
  hipDeviceProp_t prop;
  he = hipGetDeviceProperties(&prop, g_ctx.device);
  if (he != hipSuccess) return hip_fail(he, "hipGetDeviceProperties");
  g_ctx.num_cu = prop.multiProcessorCount;
  g_ctx.dim = dim;
  g_ctx.maxc = max_concurrency;
  g_ctx.seed = seed;
  try {
    for (int fid = 0; fid <= 36; ++fid) {
      // Sec. 5 defines a hybrid only where each group gets the variables its formula needs:
      // below 10 variables, and for hybrids 27 and 28 at 11 and 12 (their last group, the
      // remainder after four rounded-up shares, gets 0 or 1), the id (and any composition built
      // on it) is left out; a call for it returns the reason
      Problem p;
      try {
        p = make_tab1(fid, dim, seed);
      } catch (const std::invalid_argument &ex) {
        g_ctx.undefined[fid] = ex.what();
        continue;
      }
      int rc = register_problem(fid, std::move(p));
      if (rc != CUROB_OK) {
        free_context();
        return rc;
      }
    }
  } catch (const std::exception &ex) {
    free_context();
    return fail(CUROB_E_ARG, "%s", ex.what());
  }
  if (g_noalloc_scratch.find(g_ctx.device) == g_noalloc_scratch.end()) {
    void *ptr = nullptr;
    he = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (he != hipSuccess || ptr == nullptr) {
      free_context();
      return hip_fail(he != hipSuccess ? he : hipErrorInvalidSymbol, "locating the static scratch");
    }
    g_noalloc_scratch[g_ctx.device] = ptr;
  }
  he = hipEventCreateWithFlags(&g_ctx.scratch_done, hipEventDisableTiming);
  if (he != hipSuccess) {
    free_context();
    return hip_fail(he, "creating the scratch event");
  }
  const size_t xb = static_cast<size_t>(max_concurrency) * dim * sizeof(double);
  he = hipMalloc(&g_ctx.stage_x, xb);
  if (he == hipSuccess) he = hipMalloc(&g_ctx.stage_out, static_cast<size_t>(max_concurrency) * sizeof(double));
  if (he != hipSuccess) {
    free_context();
    return hip_fail(he, "allocating staging buffers");
  }
  g_ctx.ready = true;
  g_err.clear();
  return CUROB_OK;
}

int dispose(void) {
  if (!g_ctx.ready) return fail(CUROB_E_STATE, "nothing to dispose");
  (void)hipStreamSynchronize(g_ctx.stream);
  free_context();
  return CUROB_OK;
}

int func_evaluate(int fid, const double *d_x, int n, double *d_out) { return evaluate(PATH_F64, fid, d_x, n, d_out); }

int func_evaluatef_noalloc(int fid, const float *d_x, int n, float *d_out) {
  Entry *e = nullptr;
  int rc = check_eval_args(fid, d_x, n, d_out, &e);
  if (rc != CUROB_OK || n == 0) return rc;
  const int path = fp32_path(fid);
  hipError_t he;
  if (e->host.type == Problem::BASIC && e->dev[path].ready) {
    // the resident kernel works without scratch
    const DevProb &pb = e->dev[path].pb;
    he = launch_resident(path, pb, d_x, d_out, n, resident_shape(path, pb, n, g_ctx.num_cu), g_ctx.stream);
  } else if (e->comp.ready) {
    auto it = g_noalloc_scratch.find(g_ctx.device);
    if (it == g_noalloc_scratch.end()) return fail(CUROB_E_STATE, "no static scratch on device %d", g_ctx.device);
    CompositeScratch sc;
    if (!carve_scratch(e->comp, it->second, kNoallocScratchBytes, sc))
      return fail(CUROB_E_CAPACITY, "function id %d needs more than the %zu-byte static scratch for %d rows", fid,
                  kNoallocScratchBytes, kTileRows);
    const bool split_auto = g_ctx.mode == CUROB_MODE_SPLIT;
    he = launch_composite(path, split_auto, e->comp, d_x, d_out, n, g_ctx.num_cu, sc, g_ctx.stream);
  } else {
    return fail(CUROB_E_HIP, "function id %d has no device tables", fid);
  }
  if (he != hipSuccess) return hip_fail(he, "kernel launch");
  return CUROB_OK;
}

int func_evaluatef(int fid, const float *d_x, int n, float *d_out) { return evaluate(fp32_path(fid), fid, d_x, n, d_out); }

int h_func_evaluate(int fid, const double *h_x, int n, double *h_out) {
  return h_evaluate<double>(PATH_F64, fid, h_x, n, h_out);
}

int h_func_evaluatef(int fid, const float *h_x, int n, float *h_out) {
  return h_evaluate<float>(fp32_path(fid), fid, h_x, n, h_out);
}

int curob_de_run(int fid, int fp64, int np, double F, double CR, unsigned long long seed, void *d_pop, void *d_fit,
                 void *d_trial, void *d_ftrial, unsigned long long *d_gen, int generations) {
  Entry *e = nullptr;
  int rc = check_eval_args(fid, d_pop, np, d_fit, &e);
  if (rc != CUROB_OK) return rc;
  if (np < 4) return fail(CUROB_E_ARG, "differential evolution needs np >= 4 (got %d)", np);
  if (!d_trial || !d_ftrial || !d_gen) return fail(CUROB_E_ARG, "null pointer");
  if (!(F > 0.0 && F <= 2.0) || !(CR >= 0.0 && CR <= 1.0))
    return fail(CUROB_E_ARG, "F must be in (0, 2] and CR in [0, 1]");
  if (generations < 0) return fail(CUROB_E_ARG, "generations must be >= 0");
  const int path = fp64 ? PATH_F64 : fp32_path(fid);
  for (int g = 0; g < generations; ++g) {
    hipError_t he = launch_de_trial(fp64 != 0, d_pop, d_trial, np, g_ctx.dim, F, CR, seed, d_gen, g_ctx.stream);
    if (he != hipSuccess) return hip_fail(he, "trial vectors");
    rc = evaluate(path, fid, d_trial, np, d_ftrial);
    if (rc != CUROB_OK) return rc;
    he = launch_de_select(fp64 != 0, d_pop, d_fit, d_trial, d_ftrial, np, g_ctx.dim, d_gen, g_ctx.stream);
    if (he != hipSuccess) return hip_fail(he, "selection");
  }
  return CUROB_OK;
}

int curob_shape_key(int fid, int fp64, int n, int *key4) {
  Entry *e = nullptr;
  int rc = check_eval_args(fid, nullptr, 0, nullptr, &e);
  if (rc != CUROB_OK) return rc;
  const int path = fp64 ? PATH_F64 : fp32_path(fid);
  if (!(e->host.type == Problem::BASIC && e->dev[path].ready))
    return fail(CUROB_E_ARG, "function id %d does not run on the resident kernel (dimension <= 128)", fid);
  if (!key4) return fail(CUROB_E_ARG, "null pointer");
  const ShapeKey k = shape_key(path, e->dev[path].pb, n < 1 ? 1 : n);
  key4[0] = k.path;
  key4[1] = k.dbucket;
  key4[2] = k.fclass;
  key4[3] = k.nbucket;
  return CUROB_OK;
}

int curob_set_shape(const int *key4, int waves, int grid_per8) {
  int rc = check_ready();
  if (rc != CUROB_OK) return rc;
  if (!key4) return fail(CUROB_E_ARG, "null pointer");
  if (waves < 0 || waves > 16 || grid_per8 < 0) return fail(CUROB_E_ARG, "waves must be in 0..16, grid_per8 >= 0");
  ShapeKey k{key4[0], key4[1], key4[2], key4[3]};
  if (waves == 0) {
    erase_shape_override(k);  // back to the built-in heuristic
    return CUROB_OK;
  }
  set_shape_override(k, waves, grid_per8);
  return CUROB_OK;
}

int curob_tune(int fid, int fp64, const void *d_x, int n, void *d_out, int reps, int *best_waves, int *best_grid_per8,
               float *best_us, float *log, int log_cap, int *log_len) {
  Entry *e = nullptr;
  int rc = check_eval_args(fid, d_x, n, d_out, &e);
  if (rc != CUROB_OK) return rc;
  if (n < 1 || reps < 1) return fail(CUROB_E_ARG, "tuning needs n >= 1 and reps >= 1");
  const int path = fp64 ? PATH_F64 : fp32_path(fid);
  if (!(e->host.type == Problem::BASIC && e->dev[path].ready))
    return fail(CUROB_E_ARG, "function id %d does not run on the resident kernel (dimension <= 128)", fid);
  const DevProb &pb = e->dev[path].pb;
  const int wmax = resident_max_waves(path, pb);
  static const int kWaves[] = {1, 2, 4, 6, 8, 12, 16};
  static const int kGrid[] = {0, 4, 8, 12, 16, 24, 32};
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipError_t he = hipEventCreate(&t0);
  if (he == hipSuccess) he = hipEventCreate(&t1);
  if (he != hipSuccess) return hip_fail(he, "creating timing events");
  float best = 3.0e38f;
  int bw = 0, bg = 0, nlog = 0;
  for (int w : kWaves) {
    if (w > wmax) continue;
    for (int g : kGrid) {
      const LaunchShape ls = resident_shape_for(path, pb, n, g_ctx.num_cu, w, g);
      he = launch_resident(path, pb, d_x, d_out, n, ls, g_ctx.stream);  // warm-up
      if (he == hipSuccess) he = hipEventRecord(t0, g_ctx.stream);
      for (int r = 0; r < reps && he == hipSuccess; ++r) he = launch_resident(path, pb, d_x, d_out, n, ls, g_ctx.stream);
      if (he == hipSuccess) he = hipEventRecord(t1, g_ctx.stream);
      if (he == hipSuccess) he = hipEventSynchronize(t1);
      float ms = 0.0f;
      if (he == hipSuccess) he = hipEventElapsedTime(&ms, t0, t1);
      if (he != hipSuccess) break;
      const float us = 1000.0f * ms / static_cast<float>(reps);
      if (log && nlog < log_cap) {
        log[3 * nlog] = static_cast<float>(ls.waves);
        log[3 * nlog + 1] = static_cast<float>(g);
        log[3 * nlog + 2] = us;
        ++nlog;
      }
      if (us < best) {
        best = us;
        bw = ls.waves;
        bg = g;
      }
    }
    if (he != hipSuccess) break;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (he != hipSuccess) return hip_fail(he, "timing a candidate shape");
  set_shape_override(shape_key(path, pb, n), bw, bg);
  if (best_waves) *best_waves = bw;
  if (best_grid_per8) *best_grid_per8 = bg;
  if (best_us) *best_us = best;
  if (log_len) *log_len = nlog;
  return CUROB_OK;
}

int curob_set_stream(void *hip_stream) {
  int rc = check_ready();
  if (rc != CUROB_OK) return rc;
  g_ctx.stream = static_cast<hipStream_t>(hip_stream);
  return CUROB_OK;
}

int curob_set_mode(int mode) {
  int rc = check_ready();
  if (rc != CUROB_OK) return rc;
  if (mode < CUROB_MODE_SPLIT || mode > CUROB_MODE_SPLIT_BF16X6) return fail(CUROB_E_ARG, "unknown mode %d", mode);
  g_ctx.mode = mode;
  return CUROB_OK;
}

static int check_custom_id(int id) {
  if (id < CUROB_CUSTOM_ID_MIN || id > CUROB_CUSTOM_ID_MAX)
    return fail(CUROB_E_ARG, "custom ids must be in [%d, %d]", CUROB_CUSTOM_ID_MIN, CUROB_CUSTOM_ID_MAX);
  return CUROB_OK;
}

int curob_define_basic(int id, int base, double scale, double offset, int rotated) {
  int rc = check_ready();
  if (rc == CUROB_OK) rc = check_custom_id(id);
  if (rc != CUROB_OK) return rc;
  if (base < 0 || base > 22) return fail(CUROB_E_ARG, "base must be in 0..22");
  try {
    return register_problem(id, make_basic(base, g_ctx.dim, g_ctx.seed, static_cast<uint32_t>(id) << 8, scale, offset,
                                           rotated != 0, false));
  } catch (const std::exception &ex) {
    return fail(CUROB_E_ARG, "%s", ex.what());
  }
}

int curob_define_hybrid(int id, int ngroups, const int *bases, const double *p) {
  int rc = check_ready();
  if (rc == CUROB_OK) rc = check_custom_id(id);
  if (rc != CUROB_OK) return rc;
  if (!bases || !p) return fail(CUROB_E_ARG, "null pointer");
  try {
    return register_problem(id, make_hybrid(g_ctx.dim, g_ctx.seed, static_cast<uint32_t>(id) << 8, ngroups, bases, p));
  } catch (const std::exception &ex) {
    return fail(CUROB_E_ARG, "%s", ex.what());
  }
}

int curob_define_composition(int id, int ncomp, const int *bases, const double *sigma, const double *lambda,
                             const double *bias) {
  int rc = check_ready();
  if (rc == CUROB_OK) rc = check_custom_id(id);
  if (rc != CUROB_OK) return rc;
  if (!bases || !sigma || !lambda || !bias) return fail(CUROB_E_ARG, "null pointer");
  try {
    return register_problem(
        id, make_composition(g_ctx.dim, g_ctx.seed, static_cast<uint32_t>(id) << 8, ncomp, bases, sigma, lambda, bias));
  } catch (const std::exception &ex) {
    return fail(CUROB_E_ARG, "%s", ex.what());
  }
}

const char *curob_last_error(void) { return g_err.c_str(); }

int curob_get_problem(int fid, double *o, double *R) {
  int rc = check_ready();
  if (rc != CUROB_OK) return rc;
  auto it = g_ctx.entries.find(fid);
  if (it == g_ctx.entries.end()) return not_defined(fid);
  const Problem &p = it->second->host;
  if (p.type != Problem::BASIC) return fail(CUROB_E_FID, "id %d is not a basic function", fid);
  if (o) std::memcpy(o, p.o.data(), sizeof(double) * p.dim);
  if (R) {
    std::vector<double> d = dense_rotation(p);
    std::memcpy(R, d.data(), sizeof(double) * d.size());
  }
  return CUROB_OK;
}

int curob_get_dim(int *dim, int *max_concurrency) {
  int rc = check_ready();
  if (rc != CUROB_OK) return rc;
  if (dim) *dim = g_ctx.dim;
  if (max_concurrency) *max_concurrency = g_ctx.maxc;
  return CUROB_OK;
}

int curob_get_info(int fid, int comp, int *type, int *count, int *nseg) {
  const Problem *p = nullptr;
  int rc = find_entry(fid, &p);
  return rc != CUROB_OK ? rc : export_info(*p, comp, type, count, nseg);
}

int curob_get_structure(int fid, int comp, double *o, int *perm, int *sizes, double *blocks, int *bases,
                        double *scale, double *offset) {
  const Problem *p = nullptr;
  int rc = find_entry(fid, &p);
  return rc != CUROB_OK ? rc : export_structure(*p, comp, o, perm, sizes, blocks, bases, scale, offset);
}

int curob_get_composition(int fid, double *sigma, double *lambda, double *bias) {
  const Problem *p = nullptr;
  int rc = find_entry(fid, &p);
  return rc != CUROB_OK ? rc : export_composition(*p, sigma, lambda, bias);
}

int curob_generate_info(int fid, int dim, unsigned long long seed, int comp, int *type, int *count, int *nseg) {
  Problem p;
  int rc = generate_tab1(fid, dim, seed, p);
  return rc != CUROB_OK ? rc : export_info(p, comp, type, count, nseg);
}

int curob_generate_structure(int fid, int dim, unsigned long long seed, int comp, double *o, int *perm, int *sizes,
                             double *blocks, int *bases, double *scale, double *offset) {
  Problem p;
  int rc = generate_tab1(fid, dim, seed, p);
  return rc != CUROB_OK ? rc : export_structure(p, comp, o, perm, sizes, blocks, bases, scale, offset);
}

int curob_generate_composition(int fid, int dim, unsigned long long seed, double *sigma, double *lambda,
                               double *bias) {
  Problem p;
  int rc = generate_tab1(fid, dim, seed, p);
  return rc != CUROB_OK ? rc : export_composition(p, sigma, lambda, bias);
}

int curob_generate_basic(int fid, int dim, unsigned long long seed, double *o, double *R) {
  if (fid < 0 || fid > 22) return fail(CUROB_E_FID, "fid must be in 0..22");
  if (dim < 2) return fail(CUROB_E_ARG, "dim must be >= 2");
  Problem p = make_tab1_basic(fid, dim, seed);
  if (o) std::memcpy(o, p.o.data(), sizeof(double) * dim);
  if (R) {
    std::vector<double> d = dense_rotation(p);
    std::memcpy(R, d.data(), sizeof(double) * d.size());
  }
  return CUROB_OK;
}

}  // extern "C"
