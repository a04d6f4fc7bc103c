/*
 * curob.h -- C ABI of libcurob.so, an MI355X (gfx950) evaluator for the cuROB real-parameter
 * test functions (Ding & Tan, "A CUDA-Based Real Parameter Optimization Benchmark",
 * arXiv 1407.7737).
 *
 * Every function evaluates f(x) = f_opt + g(R (s (x - o)) + c) for whole populations of
 * candidate vectors, where g is one of the formulas of Secs. 3-4 (Tab. 1 ids 0-22), o is the
 * shifted optimum, R the three-block orthogonal rotation and s, c the scale and offset of that
 * function's definition; hybrids (Sec. 5) and compositions (Sec. 6) combine such pieces.
 *
 * Conventions for every call below.
 *  - Return value: CUROB_OK (0) or a negative CUROB_E_* code; nothing throws or aborts.
 *    curob_last_error() describes the most recent failure of the calling process.
 *  - Layout: a population is n row-major candidate vectors of `dim` contiguous elements
 *    (no padding); results are n contiguous values, one per row.
 *  - Device pointers: func_evaluate / func_evaluatef take pointers to GPU memory (Sec. 1.3,
 *    "Interface") and run asynchronously on the stream set by curob_set_stream (default: the
 *    null stream).  The h_ variants take host memory and return after the results are copied
 *    back (Sec. 1.3: wrappers of the GPU calls for CPU code).
 *  - Ownership: the caller owns x and out; the library owns all problem data it generates,
 *    and dispose() frees it.  One library context per process; calls are not thread-safe.
 *  - Sizes: 0 <= n <= max_concurrency (the capacity fixed at initialize, Sec. 1.3); n = 0 is
 *    a no-op.  A null pointer with n > 0 is CUROB_E_ARG.  x must hold n rows of exactly the
 *    `dim` given to initialize (curob_get_dim reports it); the library cannot check a raw
 *    pointer's extent.
 *  - Streams: hybrids, compositions and basic functions above 128 dimensions work through one
 *    library-owned scratch buffer.  A call of that kind issued on another stream than the
 *    previous one waits (on the device) for that previous call to finish; calls on one stream
 *    are ordered by the stream.  Under stream capture no such wait is recorded: the capturing
 *    caller keeps scratch-using calls on one stream.
 */
#ifndef CUROB_H
#define CUROB_H

#ifdef __cplusplus
extern "C" {
#endif

#define CUROB_OK 0
#define CUROB_E_STATE (-1)    /* called before initialize / after dispose / double initialize */
#define CUROB_E_ARG (-2)      /* bad dimension, count, pointer or parameter */
#define CUROB_E_FID (-3)      /* function id not defined */
#define CUROB_E_CAPACITY (-4) /* n > max_concurrency */
#define CUROB_E_HIP (-5)      /* HIP runtime failure (no device, out of memory, launch error) */

/* FP32 entry point arithmetic, chosen by curob_set_mode.  The rotation runs on the matrix
 * cores in every mode; the modes differ in how FP32 operands are represented there. */
#define CUROB_MODE_SPLIT 0        /* default: BF16 split products, x3 or x6 chosen per formula */
#define CUROB_MODE_FP32 1         /* FP32 MFMA products (the plain FP32 path) */
#define CUROB_MODE_SPLIT_BF16X3 2 /* y = hi + lo, Q = hi + lo: hi*hi + hi*lo + lo*hi, FP32 accumulate */
#define CUROB_MODE_SPLIT_BF16X6 3 /* three-term splits of y and Q, the six products of order <= 2 */

/* Tab. 1 function ids (the `fid` argument) */
enum curob_fid {
  SPHERE = 0, ELLIPSOID = 1, ELLIPTIC = 2, DISCUS = 3, CIGAR = 4, POWERS = 5, SHARPV = 6,
  STEP = 7, WEIERSTRASS = 8, GRIEWANK = 9, RASTRIGIN_U = 10, RASTRIGIN = 11, SCHAFFERSF7 = 12,
  GRIE_ROSEN = 13, ROSENBROCK = 14, SCHWEFEL_U = 15, SCHWEFEL = 16, KATSUURA = 17, LUNACEK = 18,
  ACKLEY = 19, HAPPYCAT = 20, HGBAT = 21, SCHAFFERSF6 = 22,
  HYBRID1 = 23, HYBRID2 = 24, HYBRID3 = 25, HYBRID4 = 26, HYBRID5 = 27, HYBRID6 = 28,
  COMPOSITION1 = 29, COMPOSITION2 = 30, COMPOSITION3 = 31, COMPOSITION4 = 32,
  COMPOSITION5 = 33, COMPOSITION6 = 34, COMPOSITION7 = 35, COMPOSITION8 = 36
};

/* Custom problems defined at run time take ids in [CUROB_CUSTOM_ID_MIN, CUROB_CUSTOM_ID_MAX]. */
#define CUROB_CUSTOM_ID_MIN 64
#define CUROB_CUSTOM_ID_MAX 1023

/* ---- the paper's interface (Sec. 1.3) ------------------------------------------------- */

/* Performs all set-up (Sec. 1.3 "Interface"): draws every function's optimum o uniformly in
 * [-70,70]^dim and its rotation from three random, almost equal variable groups, each block
 * an orthonormalised matrix of N(0,1) entries (Sec. 1.2), all from `seed`; uploads them to the
 * current HIP device and reserves staging for max_concurrency rows.  dim >= 2 (Sec. 1.2).
 * A Tab. 1 id whose definition leaves it undefined at this dimension is left out, and every
 * call for it returns CUROB_E_FID with the reason: the hybrids (and compositions 35 and 36)
 * below dim 10, and hybrids 27 and 28 (and composition 36, built on them) at dim 11 and 12,
 * where their last group, the remainder after four rounded-up shares (Sec. 5, Eq. (numbers)),
 * gets fewer variables than its formula needs.  Errors: CUROB_E_STATE if already initialised,
 * CUROB_E_ARG for dim < 2 or max_concurrency < 1, CUROB_E_HIP if no device or memory is
 * available. */
int initialize(int dim, int max_concurrency, unsigned long long seed);

/* Releases everything initialize and later calls allocated (Sec. 1.3).  Returns CUROB_E_STATE
 * when nothing is initialised. */
int dispose(void);

/* FP64 evaluation of function `fid` on n device-resident rows d_x (n x dim doubles), writing n
 * doubles to d_out (Sec. 1.3, func_evaluate).  Asynchronous on the library stream. */
int func_evaluate(int fid, const double *d_x, int n, double *d_out);

/* FP32 evaluation (Sec. 1.3, func_evaluatef): n x dim floats in, n floats out, device
 * pointers, asynchronous.  The rotation arithmetic follows curob_set_mode; in the default
 * CUROB_MODE_SPLIT the formulas whose FP32 value amplifies rounding of z (elliptic, discus,
 * step, Weierstrass, Schaffer F7, Griewank-Rosenbrock, rotated Schwefel, Katsuura) use the
 * six-product split, all others the three-product split. */
int func_evaluatef(int fid, const float *d_x, int n, float *d_out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): func_evaluatef with no allocation of any kind.  Same
 * arguments, arithmetic, results and errors as func_evaluatef, asynchronous on the library
 * stream.  Problems whose kernels need scratch (hybrids, compositions, basic functions above
 * 128 dimensions) take it from a static device array of CUROB_NOALLOC_SCRATCH_BYTES per device,
 * held until the process ends, in passes of as many rows as fit (at most 65536); a problem
 * whose 128-row pass does not fit is CUROB_E_CAPACITY.  Every call on a device shares that
 * device's array: calls that overlap on one device (other streams or threads) race and must
 * be serialised by the caller.  Nothing in the array needs clearing between calls: every
 * kernel writes each scratch entry it reads within the same call. */
#define CUROB_NOALLOC_SCRATCH_BYTES (32ull << 20)
int func_evaluatef_noalloc(int fid, const float *d_x, int n, float *d_out);

/* Host-pointer wrappers of the two calls above (Sec. 1.3): copy h_x to the device, evaluate,
 * copy the results to h_out and wait for them. */
int h_func_evaluate(int fid, const double *h_x, int n, double *h_out);
int h_func_evaluatef(int fid, const float *h_x, int n, float *h_out);

/* ---- extensions ----------------------------------------------------------------------- */

/* Stream for subsequent device-pointer calls (a hipStream_t; NULL = null stream). */
int curob_set_stream(void *hip_stream);

/* Rotation arithmetic of func_evaluatef: one of the CUROB_MODE_* values above. */
int curob_set_mode(int mode);

/* A basic formula `base` (0..22) under a caller-chosen transform z = R(scale (x - o)) + offset
 * (rotated != 0) or z = scale (x - o) + offset, with its own random o and R; registered as
 * custom id `id` for the current dimension.  Used, e.g., for Rastrigin at scale 1. */
int curob_define_basic(int id, int base, double scale, double offset, int rotated);

/* Hybrid function (Sec. 5, Eq. (hybrid)): y = x - o is permuted by a random S and cut into
 * ngroups consecutive groups of sizes n_i = ceil(p_i dim) (i < ngroups) and the remainder
 * (Eq. (numbers)); group i contributes g_{base_i}(R_i (s_i z^i) + c_i) at dimension n_i, with
 * its own dense random rotation R_i.  1 <= ngroups <= 8.  Every n_i must be >= 1, and >= 2 for
 * the formulas that divide by n - 1 (elliptic 2, different powers 5, Schaffer F7 12); other
 * sizes are CUROB_E_ARG. */
int curob_define_hybrid(int id, int ngroups, const int *bases, const double *p);

/* Composition function (Sec. 6, Eqs. (composition) and (weight)): ncomp (1..8) basic
 * components, each with its own random optimum o^i and rotation, blended with weights
 * w_i = exp(-d_i^2 / (2 dim sigma_i^2)) / d_i, d_i = |x - o^i|, normalised to sum to one
 * (one-hot at x = o^i): F = sum_i omega_i (lambda_i G_i(x) + bias_i) + f_opt. */
int curob_define_composition(int id, int ncomp, const int *bases, const double *sigma,
                             const double *lambda, const double *bias);

/* Message for the last failure of any call ("" if none). */
const char *curob_last_error(void);

/* Generated problem data, for checks: the shift o (dim doubles) and the dense rotation R
 * (dim x dim doubles, row-major; the identity when the function is unrotated).  Either
 * pointer may be NULL.  Works for ids 0..22 and custom basic ids. */
int curob_get_problem(int fid, double *o, double *R);

/* Host-only generator entry point (no device needed): the same o and R that initialize(dim,
 * ..., seed) produces for basic function `fid` (0..22). */
int curob_generate_basic(int fid, int dim, unsigned long long seed, double *o, double *R);

/* The dimension and capacity given to initialize.  CUROB_E_STATE before initialize. */
int curob_get_dim(int *dim, int *max_concurrency);

/* ---- problem structure export (for checks against an independent implementation) ---------
 * A problem is described part by part: comp < 0 names the problem itself, comp = 0..N-1 a
 * component of a composition (CUROB_E_ARG for other problems or out of range).
 *
 * curob_get_info: *type = 0 basic, 1 hybrid, 2 composition; *count = rotation blocks (basic:
 *   the up to three variable groups of Sec. 1.2, 0 when unrotated; hybrid: its N groups, Sec. 5)
 *   or components (composition, Sec. 6); *nseg = formula segments (basic 1, hybrid N, composition
 *   0).  Any output pointer may be NULL.
 * curob_get_structure: for a basic or hybrid part: o (dim doubles, the shift, original variable
 *   order); perm (dim ints: packed position -> original variable, 0-based; the permutation S of
 *   Sec. 5 Eq. (hybrid) for hybrids, the group order of Sec. 1.2 for basic functions); sizes
 *   (count ints, block sizes n_k in packed order); blocks (sum n_k^2 doubles: each n_k x n_k
 *   orthonormal block row-major, one after another, so z_a = sum_b Q[a][b] (s y_perm[off+b]) + c
 *   within a block); bases, scale, offset (nseg entries: Tab. 1 formula id, s and c of each
 *   segment).  Any pointer may be NULL; non-NULL ones must hold the sizes above.  A composition
 *   itself (comp < 0) is CUROB_E_ARG: name a component.
 * curob_get_composition: sigma_i, lambda_i and bias_i of a composition (count values each,
 *   Sec. 6 Eq. (composition)); CUROB_E_ARG for other problems.
 * These read the problem registered under fid in the initialised library (CUROB_E_STATE before
 * initialize, CUROB_E_FID for an unknown id).  The curob_generate_* forms generate Tab. 1
 * problem fid (0..36) for (dim, seed) on the host instead, exactly as initialize(dim, ..., seed)
 * would, with no device and no library state (CUROB_E_ARG for dim < 2 and for the ids that
 * initialize leaves undefined at dim, with the reason). */
int curob_get_info(int fid, int comp, int *type, int *count, int *nseg);
int curob_get_structure(int fid, int comp, double *o, int *perm, int *sizes, double *blocks, int *bases,
                        double *scale, double *offset);
int curob_get_composition(int fid, double *sigma, double *lambda, double *bias);
int curob_generate_info(int fid, int dim, unsigned long long seed, int comp, int *type, int *count, int *nseg);
int curob_generate_structure(int fid, int dim, unsigned long long seed, int comp, double *o, int *perm, int *sizes,
                             double *blocks, int *bases, double *scale, double *offset);
int curob_generate_composition(int fid, int dim, unsigned long long seed, double *sigma, double *lambda,
                               double *bias);

/* ---- an optimiser in the loop: differential evolution on the GPU ------------------------
 * The paper's motivating use (Sec. 1; Sec. 2 evaluates 50 candidates per call): an optimiser
 * running on the GPU calls the evaluation interface every generation.  curob_de_run enqueues
 * `generations` generations of DE/rand/1/bin on the library stream, each: trial vectors from
 * the population, their evaluation through func_evaluate (fp64 != 0) or func_evaluatef, and
 * greedy selection (a trial replaces its target when its value is not larger), then the
 * device generation counter *d_gen advances by one.  Nothing is allocated, copied or cleared,
 * so the call can be captured in a HIP graph; replays continue from the counter.
 * Trial of individual i in generation g: r1, r2, r3 distinct and != i, a forced position
 * j_rand, and for each variable j: t_j = clamp(fma(F, x_r2j - x_r3j, x_r1j), -100, 100) if
 * u_j < CR or j = j_rand, else x_ij (FP64 or FP32 arithmetic as the population).  Random draw k
 * is SplitMix64's output for state seed + (k + 1) 0x9E3779B97F4A7C15 with k = (g np + i)(dim + 4)
 * + slot; slots 0, 1, 2 pick r1, r2, r3 (each the v-th allowed index in increasing order,
 * v = draw mod (number allowed)), slot 3 gives j_rand = draw mod dim, slot 4 + j gives
 * u_j = (draw >> 11) 2^-53.
 * Buffers (device, caller-owned, of the population's type): d_pop np x dim, d_fit np (the
 * values of d_pop, e.g. from func_evaluate[f]), d_trial np x dim and d_ftrial np (work space),
 * d_gen one unsigned 64-bit generation counter.  4 <= np <= max_concurrency, 0 < F <= 2,
 * 0 <= CR <= 1; otherwise CUROB_E_ARG (CUROB_E_CAPACITY for np > max_concurrency). */
int curob_de_run(int fid, int fp64, int np, double F, double CR, unsigned long long seed, void *d_pop, void *d_fit,
                 void *d_trial, void *d_ftrial, unsigned long long *d_gen, int generations);

/* ---- autotuned launch shapes of the single-call kernel ------------------------------------
 * Basic functions up to 128 dimensions run on one persistent kernel whose launch shape -- waves
 * (16-row column blocks) per workgroup and workgroups per 8 CUs -- is chosen per key (path,
 * D bucket, formula class, row-count bucket): D buckets 0..4 for dim <= 16, 32, 64, 96, 128;
 * the class is 2 * (formula family) + rotated; the row bucket is floor(log2 n) in 4..24; the
 * path is that of func_evaluate (fp64 != 0) or of func_evaluatef in the current mode.  Keys
 * without an entry use the built-in heuristic (as many waves as the LDS holds, at most
 * occupancy x CUs workgroups).  Entries live until dispose.
 *
 * curob_shape_key: the four key values for function fid, path and n rows (CUROB_E_ARG when the
 *   function does not run on that kernel, i.e. dim > 128, hybrids, compositions).
 * curob_set_shape: installs (waves 1..16, grid_per8 >= 0; 0 = occupancy x CUs) for a key, e.g.
 *   from a cache of earlier tuning; waves = 0 removes the key's entry.  Waves are clamped to what
 *   the LDS allows for the problem at launch.
 * curob_tune: times every candidate (waves {1, 2, 4, 6, 8, 12, 16} up to the LDS limit x
 *   grid_per8 {0, 4, 8, 12, 16, 24, 32}) with `reps` launches each (after one warm-up) on the
 *   caller's device buffers d_x (n rows) and d_out, on the library stream (waits for it), and
 *   installs the fastest for the key of (fid, path, n).  Outputs: the best shape and its time
 *   per launch in microseconds; if log != NULL, up to log_cap triples (waves, grid_per8, us), one
 *   per candidate timed, and their count in *log_len.  d_out is overwritten. */
int curob_shape_key(int fid, int fp64, int n, int *key4);
int curob_set_shape(const int *key4, int waves, int grid_per8);
int curob_tune(int fid, int fp64, const void *d_x, int n, void *d_out, int reps, int *best_waves, int *best_grid_per8,
               float *best_us, float *log, int log_cap, int *log_len);

/* ---- batched populations (one persistent launch, replayed as a HIP graph) --------------- */

typedef struct curob_batch curob_batch;

/* Plans k populations evaluated by one persistent launch (needs an initialised library; the
 * launches go to the library stream).  Population i has counts[i] >= 0 rows of dims[i]
 * (2..128) FP32 elements and is Tab. 1 function fids[i] (0..22) with that function's
 * transform (Secs. 3-4), its shift and rotation drawn like a custom problem with id
 * 2048 + i (the key (2048 + i) << 8 of the generator streams, Sec. 1.2) at dimension dims[i].
 * Arithmetic: the FP32 split path, three or six BF16 products per formula as the default mode
 * picks.  The plan, device tables and the HIP graph are owned by *out; the default launch
 * shape is two waves per workgroup, two row groups per item, two workgroups per CU.
 * Errors: CUROB_E_STATE before initialize, CUROB_E_FID for a fid outside 0..22, CUROB_E_ARG for
 * k outside 1..65536, a dimension outside 2..128 or a negative count, CUROB_E_HIP. */
int curob_batch_create(int k, const int *fids, const int *dims, const int *counts,
                       unsigned long long seed, curob_batch **out);

/* Points the batch at device buffers: d_xs[i] holds counts[i] x dims[i] floats (row-major),
 * d_outs[i] receives counts[i] floats; host arrays of k device pointers (may be NULL where
 * counts[i] = 0).  Waits for the library stream, then copies the pointer tables to the
 * device; the first bind captures the graph, later binds reuse it. */
int curob_batch_bind(curob_batch *b, const float *const *d_xs, float *const *d_outs);

/* Replays the captured graph on the library stream (asynchronous).  CUROB_E_STATE before the
 * first bind. */
int curob_batch_run(curob_batch *b);

/* The same launch without the graph (for timing the graph's benefit). */
int curob_batch_run_direct(curob_batch *b);

/* Sets the launch shape: waves per workgroup (1..4, and the LDS of the largest population
 * must fit), row groups of 32 rows per work item, workgroups (clamped to the item count).
 * Re-plans the schedule and re-captures the graph. */
int curob_batch_configure(curob_batch *b, int waves, int groups_per_item, int grid);

/* The current launch shape and the number of work items. */
int curob_batch_shape(const curob_batch *b, int *waves, int *groups_per_item, int *grid, int *nitems);

/* Autotuner: times every candidate shape (waves {1,2,4} x groups per item {1,2,4,8} x waves x
 * workgroups {CUs/2, CUs, 2 CUs, 4 CUs}) with `reps` launches each on the bound buffers,
 * keeps the fastest and re-captures the graph; *best_us receives its time per launch.
 * Needs a bound batch (CUROB_E_STATE otherwise). */
int curob_batch_tune(curob_batch *b, int reps, float *best_us);

/* Frees a batch (after waiting for the library stream).  NULL is ignored. */
int curob_batch_destroy(curob_batch *b);

/* ---- Measured peaks (for benchmarks that report a roofline) ---------------------------------
 * Not part of the evaluation interface: callers are benchmarks that state a measured peak
 * beside the nominal one.  Both run on the library stream, wait for it, and report the
 * fastest of `reps` timed launches (one untimed warm-up first).  Need an initialised library
 * (CUROB_E_STATE otherwise); they allocate and free a 16-byte device buffer per call.
 *
 * curob_probe_read: reads every 16-byte word of the device buffer d_buf (bytes: a positive
 *   multiple of 16, d_buf 16-byte aligned, else CUROB_E_ARG) once per launch on a grid of
 *   8 workgroups per CU; *gbs = bytes / time in GB/s.  The buffer is only read.
 * curob_probe_mfma_bf16: four 4-wave workgroups per CU each issue 4 x 4096 dense 16x16x32
 *   BF16 MFMAs per wave in four independent chains; *tflops = 16384 flops x MFMAs / time. */
int curob_probe_read(const void *d_buf, unsigned long long bytes, int reps, double *gbs);
int curob_probe_mfma_bf16(int reps, double *tflops);

#ifdef __cplusplus
}
#endif

#endif /* CUROB_H */
