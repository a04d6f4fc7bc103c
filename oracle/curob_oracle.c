/*
 * curob_oracle.c -- plain, slow, FP64 CPU oracle for the cuROB test-function suite
 * (Ding & Tan, "A CUDA-Based Real Parameter Optimization Benchmark", arXiv 1407.7737).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference for the GPU library in
 * paper_1407_7737_amd/.  It shares no code, header, table or helper with that library and
 * must never be linked into it.  Only tests/, __graft_entry__.smoke() and the cpu_baseline
 * leg of bench.py load it.
 *
 * Everything is computed in IEEE double with plain loops: y = s*(x - o), z = R*y + c with a
 * materialised dense D x D rotation, then the formula g(z) written out term by term, then the
 * bias f_opt.  No blocking, no fusion, no reordering beyond what each definition states.
 *
 * Problem data (shift vector, variable groups, rotation blocks) are drawn from SplitMix64
 * (Steele, Lea & Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014), with
 * normals from the Marsaglia polar method and the orthonormal blocks from classical
 * Gram-Schmidt applied twice (CGS2).  The GPU library implements the same published
 * generator on its own, and orthonormalises with Householder QR instead, so the two agree
 * only because the orthonormal factor with positive diagonal is unique.
 *
 * Parity status: every formula is pinned by tests/test_oracle_*.py against closed forms,
 * invariants, special cases and D=2 brute force, except where noted "parity unpinned" below
 * (agreement with the original cuROB binaries and data, which the paper does not provide).
 * The transcribed constants -- each function's scale, offset and rotation flag (Secs. 3-4),
 * the hybrid tables (Sec. 5) and the composition tables (Sec. 6) -- are pinned against
 * fixtures of the printed values, element by element and through the values they produce.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXC 16
#define ORC_PI 3.14159265358979323846
#define ORC_E 2.71828182845904523536

/* ------------------------------------------------------------------------------------------
 * SplitMix64 (published definition): a Weyl sequence with increment 0x9E3779B97F4A7C15,
 * each state passed through the 64-bit finaliser below.
 * ---------------------------------------------------------------------------------------- */
static uint64_t orc_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

typedef struct {
  uint64_t state;
  int have_spare;
  double spare;
} orc_rng;

/* One independent stream per (seed, dimension, problem key, purpose).
 * purpose 0 = shift vector, 1 = variable permutation, 2 = rotation entries. */
static void orc_rng_open(orc_rng *g, uint64_t seed, int dim, uint32_t key, uint32_t purpose) {
  uint64_t tag = ((uint64_t)key << 32) ^ ((uint64_t)purpose << 24) ^ (uint64_t)(uint32_t)dim;
  g->state = orc_mix64(seed ^ orc_mix64(tag));
  g->have_spare = 0;
  g->spare = 0.0;
}

static uint64_t orc_next(orc_rng *g) {
  g->state += 0x9E3779B97F4A7C15ULL;
  return orc_mix64(g->state);
}

/* uniform on [0,1): the top 53 bits scaled by 2^-53 */
static double orc_uniform(orc_rng *g) { return (double)(orc_next(g) >> 11) * 0x1.0p-53; }

/* standard normal by the Marsaglia polar method; the second variate of each pair is kept */
static double orc_normal(orc_rng *g) {
  if (g->have_spare) {
    g->have_spare = 0;
    return g->spare;
  }
  double u, v, s;
  do {
    u = 2.0 * orc_uniform(g) - 1.0;
    v = 2.0 * orc_uniform(g) - 1.0;
    s = u * u + v * v;
  } while (s >= 1.0 || s == 0.0);
  double m = sqrt(-2.0 * log(s) / s);
  g->spare = v * m;
  g->have_spare = 1;
  return u * m;
}

/* ------------------------------------------------------------------------------------------
 * Problem construction (General Setup, Sec. 1.2)
 * ---------------------------------------------------------------------------------------- */

/* x_opt drawn uniformly from [-70,70]^D (Sec. 1.2, "x_opt"). */
static void orc_make_shift(uint64_t seed, int dim, uint32_t key, double *o) {
  orc_rng g;
  orc_rng_open(&g, seed, dim, key, 0);
  for (int j = 0; j < dim; ++j) o[j] = -70.0 + 140.0 * orc_uniform(&g);
}

/* A uniformly random permutation of 0..D-1 by Fisher-Yates (random split of the variables,
 * Sec. 1.2 "Rotation Matrix"; hybrid permutation S, Sec. 5). */
static void orc_make_perm(uint64_t seed, int dim, uint32_t key, int *perm) {
  orc_rng g;
  orc_rng_open(&g, seed, dim, key, 1);
  for (int j = 0; j < dim; ++j) perm[j] = j;
  for (int i = dim - 1; i >= 1; --i) {
    int j = (int)(orc_next(&g) % (uint64_t)(i + 1));
    int t = perm[i];
    perm[i] = perm[j];
    perm[j] = t;
  }
}

/* Orthonormalise the columns of the n x n row-major matrix A in place by classical
 * Gram-Schmidt with one full re-orthogonalisation pass (CGS2). */
static void orc_cgs2(int n, double *A) {
  double *v = (double *)malloc(sizeof(double) * (size_t)n);
  double *c = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  for (int j = 0; j < n; ++j) {
    for (int r = 0; r < n; ++r) v[r] = A[r * n + j];
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = 0; i < j; ++i) {
        double d = 0.0;
        for (int r = 0; r < n; ++r) d += A[r * n + i] * v[r];
        c[i] = d;
      }
      for (int i = 0; i < j; ++i)
        for (int r = 0; r < n; ++r) v[r] -= c[i] * A[r * n + i];
    }
    double nrm = 0.0;
    for (int r = 0; r < n; ++r) nrm += v[r] * v[r];
    nrm = sqrt(nrm);
    for (int r = 0; r < n; ++r) A[r * n + j] = v[r] / nrm;
  }
  free(v);
  free(c);
}

/* Draw one n x n block: N(0,1) entries row-major, then CGS2 on its columns (Sec. 1.2). */
static void orc_draw_block(orc_rng *g, int n, double *Q) {
  for (int k = 0; k < n * n; ++k) Q[k] = orc_normal(g);
  orc_cgs2(n, Q);
}

/* The three (almost) equal variable groups of Sec. 1.2: floor(D/3) each, the first D mod 3
 * groups one larger; empty groups (D < 3) are dropped. */
static int orc_group_sizes(int dim, int *sizes) {
  int ng = 0;
  for (int k = 0; k < 3; ++k) {
    int nk = dim / 3 + (k < dim % 3 ? 1 : 0);
    if (nk > 0) sizes[ng++] = nk;
  }
  return ng;
}

/* Dense rotation R (D x D, row-major) assembled from the group blocks: for group k holding
 * original variables S_k[0..n_k-1], R[S_k[a]][S_k[b]] = Q_k[a][b], zero across groups. */
static void orc_make_rotation(uint64_t seed, int dim, uint32_t key, double *R) {
  int *perm = (int *)malloc(sizeof(int) * (size_t)dim);
  int sizes[3];
  orc_make_perm(seed, dim, key, perm);
  int ng = orc_group_sizes(dim, sizes);
  orc_rng g;
  orc_rng_open(&g, seed, dim, key, 2);
  memset(R, 0, sizeof(double) * (size_t)dim * (size_t)dim);
  int off = 0;
  for (int k = 0; k < ng; ++k) {
    int n = sizes[k];
    double *Q = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
    orc_draw_block(&g, n, Q);
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) R[(size_t)perm[off + a] * dim + perm[off + b]] = Q[a * n + b];
    free(Q);
    off += n;
  }
  free(perm);
}

/* ------------------------------------------------------------------------------------------
 * Per-function transform of Tab. 1 functions 0..22: z = R(s*(x - o)) + c, R optional.
 * The scale s and offset c are read off each function's "where" clause.
 * ---------------------------------------------------------------------------------------- */
typedef struct {
  double s, c;
  int rotated;
} orc_xform_t;

static const orc_xform_t ORC_XF[23] = {
    {1.0, 0.0, 1},      /*  0 Sphere, Sec. 3.1 */
    {1.0, 0.0, 1},      /*  1 Ellipsoid, Sec. 3.2 */
    {1.0, 0.0, 1},      /*  2 High Conditioned Elliptic, Sec. 3.3 */
    {1.0, 0.0, 1},      /*  3 Discus, Sec. 3.4 */
    {1.0, 0.0, 1},      /*  4 Bent Cigar, Sec. 3.5 */
    {0.01, 0.0, 1},     /*  5 Different Powers, Sec. 3.6 */
    {1.0, 0.0, 1},      /*  6 Sharp Valley, Sec. 3.7 */
    {1.0, 0.0, 1},      /*  7 Step, Sec. 4.1 */
    {0.005, 0.0, 1},    /*  8 Weierstrass, Sec. 4.2 */
    {6.0, 0.0, 1},      /*  9 Griewank, Sec. 4.3 */
    {0.0512, 0.0, 0},   /* 10 Shifted Rastrigin (no rotation), Sec. 4.4 */
    {0.0512, 0.0, 1},   /* 11 Rotated Rastrigin, Sec. 4.5 */
    {1.0, 0.0, 1},      /* 12 Schaffer's F7, Sec. 4.6 */
    {0.05, 1.0, 1},     /* 13 Expanded Griewank plus Rosenbrock, Sec. 4.7 */
    {0.02048, 1.0, 1},  /* 14 Rosenbrock, Sec. 4.8 */
    {10.0, 0.0, 0},     /* 15 Modified Schwefel (no rotation), Sec. 4.9 */
    {10.0, 0.0, 1},     /* 16 Rotated Modified Schwefel, Sec. 4.10 */
    {0.05, 0.0, 1},     /* 17 Katsuura, Sec. 4.11 */
    {0.1, 2.5, 1},      /* 18 Lunacek bi-Rastrigin, Sec. 4.12 (offset read as outside R) */
    {1.0, 0.0, 1},      /* 19 Ackley, Sec. 4.13 */
    {0.05, -1.0, 1},    /* 20 HappyCat, Sec. 4.14 */
    {0.05, -1.0, 1},    /* 21 HGBat, Sec. 4.15 */
    {1.0, 0.0, 1},      /* 22 Expanded Schaffer's F6, Sec. 4.16 */
};

/* ------------------------------------------------------------------------------------------
 * The basic formulas g(z) of Secs. 3 and 4, on a vector z of length D (1-based i in the
 * paper is i+1 here).  Each returns the value before the bias f_opt.
 * ---------------------------------------------------------------------------------------- */

/* Sec. 3.1: sum z_i^2 */
static double g_sphere(int D, const double *z) {
  double f = 0.0;
  for (int i = 0; i < D; ++i) f += z[i] * z[i];
  return f;
}

/* Sec. 3.2: sum i * z_i^2 */
static double g_ellipsoid(int D, const double *z) {
  double f = 0.0;
  for (int i = 0; i < D; ++i) f += (double)(i + 1) * z[i] * z[i];
  return f;
}

/* Sec. 3.3: sum (10^6)^((i-1)/(D-1)) z_i^2 */
static double g_elliptic(int D, const double *z) {
  double f = 0.0;
  for (int i = 0; i < D; ++i) f += pow(1.0e6, (double)i / (double)(D - 1)) * z[i] * z[i];
  return f;
}

/* Sec. 3.4: 10^6 z_1^2 + sum_{i>=2} z_i^2 */
static double g_discus(int D, const double *z) {
  double f = 1.0e6 * z[0] * z[0];
  for (int i = 1; i < D; ++i) f += z[i] * z[i];
  return f;
}

/* Sec. 3.5: z_1^2 + 10^6 sum_{i>=2} z_i^2 */
static double g_cigar(int D, const double *z) {
  double t = 0.0;
  for (int i = 1; i < D; ++i) t += z[i] * z[i];
  return z[0] * z[0] + 1.0e6 * t;
}

/* Sec. 3.6: sqrt(sum |z_i|^(2 + 4(i-1)/(D-1))) */
static double g_powers(int D, const double *z) {
  double f = 0.0;
  for (int i = 0; i < D; ++i) f += pow(fabs(z[i]), 2.0 + 4.0 * (double)i / (double)(D - 1));
  return sqrt(f);
}

/* Sec. 3.7: z_1^2 + 100 sqrt(sum_{i>=2} z_i^2)  (the printed first term "z_i^2" read as z_1^2) */
static double g_sharpv(int D, const double *z) {
  double t = 0.0;
  for (int i = 1; i < D; ++i) t += z[i] * z[i];
  return z[0] * z[0] + 100.0 * sqrt(t);
}

/* Sec. 4.1: sum floor(z_i + 0.5)^2 */
static double g_step(int D, const double *z) {
  double f = 0.0;
  for (int i = 0; i < D; ++i) {
    double r = floor(z[i] + 0.5);
    f += r * r;
  }
  return f;
}

/* Sec. 4.2: sum_i sum_{k=0..20} a^k cos(2 pi b^k (z_i + 0.5)) - D sum_k a^k cos(2 pi b^k 0.5),
 * a = 0.5, b = 3 */
static double g_weierstrass(int D, const double *z) {
  double f = 0.0;
  for (int i = 0; i < D; ++i)
    for (int k = 0; k <= 20; ++k) f += pow(0.5, k) * cos(2.0 * ORC_PI * pow(3.0, k) * (z[i] + 0.5));
  double c = 0.0;
  for (int k = 0; k <= 20; ++k) c += pow(0.5, k) * cos(2.0 * ORC_PI * pow(3.0, k) * 0.5);
  return f - (double)D * c;
}

/* Sec. 4.3: sum z_i^2/4000 - prod cos(z_i/sqrt(i)) + 1 */
static double g_griewank(int D, const double *z) {
  double s = 0.0, p = 1.0;
  for (int i = 0; i < D; ++i) {
    s += z[i] * z[i] / 4000.0;
    p *= cos(z[i] / sqrt((double)(i + 1)));
  }
  return s - p + 1.0;
}

/* Sec. 4.4: sum (z_i^2 - 10 cos(2 pi z_i)) + 10 D */
static double g_rastrigin_u(int D, const double *z) {
  double f = 0.0;
  for (int i = 0; i < D; ++i) f += z[i] * z[i] - 10.0 * cos(2.0 * ORC_PI * z[i]);
  return f + 10.0 * (double)D;
}

/* Sec. 4.5: sum (z_i^2 - 10 cos(2 pi z_i) + 10) */
static double g_rastrigin(int D, const double *z) {
  double f = 0.0;
  for (int i = 0; i < D; ++i) f += z[i] * z[i] - 10.0 * cos(2.0 * ORC_PI * z[i]) + 10.0;
  return f;
}

/* Sec. 4.6: ((1/(D-1)) sum_{i<D} (1 + sin^2(50 w_i^0.2)) sqrt(w_i))^2,
 * w_i = sqrt(z_i^2 + z_{i+1}^2) */
static double g_schaffer_f7(int D, const double *z) {
  double t = 0.0;
  for (int i = 0; i + 1 < D; ++i) {
    double w = sqrt(z[i] * z[i] + z[i + 1] * z[i + 1]);
    double sn = sin(50.0 * pow(w, 0.2));
    t += (1.0 + sn * sn) * sqrt(w);
  }
  t /= (double)(D - 1);
  return t * t;
}

/* Sec. 4.7 helpers: g2 (Rosenbrock pair) and g3 (one-dimensional Griewank) */
static double g2_rosen(double x, double y) { return 100.0 * (x * x - y) * (x * x - y) + (x - 1.0) * (x - 1.0); }
static double g3_griew(double x) { return x * x / 4000.0 - cos(x) + 1.0; }

/* Sec. 4.7: sum_{i<D} g3(g2(z_i, z_{i+1})) + g3(g2(z_D, z_1)) */
static double g_grie_rosen(int D, const double *z) {
  double f = 0.0;
  for (int i = 0; i + 1 < D; ++i) f += g3_griew(g2_rosen(z[i], z[i + 1]));
  return f + g3_griew(g2_rosen(z[D - 1], z[0]));
}

/* Sec. 4.8: sum_{i<D} 100 (z_i^2 - z_{i+1})^2 + (z_i - 1)^2 */
static double g_rosenbrock(int D, const double *z) {
  double f = 0.0;
  for (int i = 0; i + 1 < D; ++i) {
    double a = z[i] * z[i] - z[i + 1];
    double b = z[i] - 1.0;
    f += 100.0 * a * a + b * b;
  }
  return f;
}

/* Sec. 4.9, Eq. (basic_schwefel): the three-branch g1 with mod taken on positive arguments */
static double g1_schwefel(double w, int D) {
  if (fabs(w) <= 500.0) return w * sin(sqrt(fabs(w)));
  if (w > 500.0) {
    double m = fmod(w, 500.0);
    return (500.0 - m) * sin(sqrt(500.0 - m)) - (w - 500.0) * (w - 500.0) / (10000.0 * (double)D);
  }
  double m = fmod(-w, 500.0);
  return (m - 500.0) * sin(sqrt(500.0 - m)) - (w + 500.0) * (w + 500.0) / (10000.0 * (double)D);
}

/* Secs. 4.9/4.10: 418.9829 D - sum g1(z_i + 420.9687462275036) */
static double g_schwefel(int D, const double *z) {
  double t = 0.0;
  for (int i = 0; i < D; ++i) t += g1_schwefel(z[i] + 420.9687462275036, D);
  return 418.9829 * (double)D - t;
}

/* Sec. 4.11: (10/D^2) prod (1 + i sum_{j=1..32} |2^j z_i - [2^j z_i]| / 2^j)^(10/D^1.2) - 10/D^2 */
static double g_katsuura(int D, const double *z) {
  double p = 1.0;
  double ex = 10.0 / pow((double)D, 1.2);
  for (int i = 0; i < D; ++i) {
    double t = 0.0;
    for (int j = 1; j <= 32; ++j) {
      double q = pow(2.0, j) * z[i];
      t += fabs(q - nearbyint(q)) / pow(2.0, j);
    }
    p *= pow(1.0 + (double)(i + 1) * t, ex);
  }
  double c = 10.0 / ((double)D * (double)D);
  return c * p - c;
}

/* Sec. 4.12: min(sum (z_i - mu1)^2, d D + s sum (z_i - mu2)^2) + 10 (D - sum cos(2 pi (z_i - mu1))),
 * mu1 = 2.5, mu2 = -2.5, d = 1, s = 0.9 */
static double g_lunacek(int D, const double *z) {
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = 0; i < D; ++i) {
    a += (z[i] - 2.5) * (z[i] - 2.5);
    b += (z[i] + 2.5) * (z[i] + 2.5);
    c += cos(2.0 * ORC_PI * (z[i] - 2.5));
  }
  double second = 1.0 * (double)D + 0.9 * b;
  return (a < second ? a : second) + 10.0 * ((double)D - c);
}

/* Sec. 4.13: -20 exp(-0.2 sqrt(mean z^2)) - exp(mean cos(2 pi z)) + 20 + e  (formula on z) */
static double g_ackley(int D, const double *z) {
  double s2 = 0.0, sc = 0.0;
  for (int i = 0; i < D; ++i) {
    s2 += z[i] * z[i];
    sc += cos(2.0 * ORC_PI * z[i]);
  }
  return -20.0 * exp(-0.2 * sqrt(s2 / (double)D)) - exp(sc / (double)D) + 20.0 + ORC_E;
}

/* Sec. 4.14: |sum z^2 - D|^0.25 + (0.5 sum z^2 + sum z)/D + 0.5 */
static double g_happycat(int D, const double *z) {
  double s2 = 0.0, s1 = 0.0;
  for (int i = 0; i < D; ++i) {
    s2 += z[i] * z[i];
    s1 += z[i];
  }
  return pow(fabs(s2 - (double)D), 0.25) + (0.5 * s2 + s1) / (double)D + 0.5;
}

/* Sec. 4.15: |(sum z^2)^2 - (sum z)^2|^0.5 + (0.5 sum z^2 + sum z)/D + 0.5 */
static double g_hgbat(int D, const double *z) {
  double s2 = 0.0, s1 = 0.0;
  for (int i = 0; i < D; ++i) {
    s2 += z[i] * z[i];
    s1 += z[i];
  }
  return pow(fabs(s2 * s2 - s1 * s1), 0.5) + (0.5 * s2 + s1) / (double)D + 0.5;
}

/* Sec. 4.16: g4(x,y) = (sin^2(sqrt(x^2+y^2)) - 0.5)/(1 + 0.001 (x^2+y^2))^2 + 0.5 */
static double g4_schaffer(double x, double y) {
  double r2 = x * x + y * y;
  double sn = sin(sqrt(r2));
  double den = 1.0 + 0.001 * r2;
  return (sn * sn - 0.5) / (den * den) + 0.5;
}

/* Sec. 4.16: sum_{i<D} g4(z_i, z_{i+1}) + g4(z_D, z_1) */
static double g_schaffer_f6(int D, const double *z) {
  double f = 0.0;
  for (int i = 0; i + 1 < D; ++i) f += g4_schaffer(z[i], z[i + 1]);
  return f + g4_schaffer(z[D - 1], z[0]);
}

typedef double (*orc_g_fn)(int, const double *);
static const orc_g_fn ORC_G[23] = {
    g_sphere,    g_ellipsoid,   g_elliptic,  g_discus,     g_cigar,      g_powers,
    g_sharpv,    g_step,        g_weierstrass, g_griewank, g_rastrigin_u, g_rastrigin,
    g_schaffer_f7, g_grie_rosen, g_rosenbrock, g_schwefel, g_schwefel,   g_katsuura,
    g_lunacek,   g_ackley,      g_happycat,  g_hgbat,      g_schaffer_f6,
};

/* ------------------------------------------------------------------------------------------
 * Problems: basic (one formula), hybrid (Sec. 5) and composition (Sec. 6)
 * ---------------------------------------------------------------------------------------- */
enum { ORC_BASIC = 0, ORC_HYBRID = 1, ORC_COMPOSITION = 2 };

typedef struct orc_problem {
  int kind, dim;
  double fopt;
  /* basic */
  int base;
  double s, c;
  double *o;  /* D */
  double *R;  /* D x D dense, NULL = identity */
  /* hybrid */
  int ngroups;
  int gbase[ORC_MAXC];
  int gsize[ORC_MAXC];
  int *perm;            /* S, D entries */
  double *gR[ORC_MAXC]; /* n_i x n_i */
  /* composition */
  int ncomp;
  double sigma[ORC_MAXC], lambda[ORC_MAXC], cbias[ORC_MAXC];
  struct orc_problem *comp[ORC_MAXC];
} orc_problem;

void orc_problem_free(orc_problem *p);

static orc_problem *orc_alloc(int kind, int dim) {
  orc_problem *p = (orc_problem *)calloc(1, sizeof(orc_problem));
  p->kind = kind;
  p->dim = dim;
  p->fopt = 100.0; /* Tab. 1 footer: f_opt = 100 for every function */
  return p;
}

/* Basic problem with explicit transform; key selects the independent random streams. */
static orc_problem *orc_basic_keyed(int base, int dim, uint64_t seed, uint32_t key, double s, double c,
                                    int rotated, int origin_optimum) {
  if (base < 0 || base > 22 || dim < 2) return NULL;
  orc_problem *p = orc_alloc(ORC_BASIC, dim);
  p->base = base;
  p->s = s;
  p->c = c;
  p->o = (double *)malloc(sizeof(double) * (size_t)dim);
  if (origin_optimum)
    memset(p->o, 0, sizeof(double) * (size_t)dim);
  else
    orc_make_shift(seed, dim, key, p->o);
  if (rotated) {
    p->R = (double *)malloc(sizeof(double) * (size_t)dim * (size_t)dim);
    orc_make_rotation(seed, dim, key, p->R);
  }
  return p;
}

/* Tab. 1 function `fid` (0..22) with its own transform. */
orc_problem *orc_problem_basic(int fid, int dim, uint64_t seed) {
  if (fid < 0 || fid > 22) return NULL;
  const orc_xform_t *t = &ORC_XF[fid];
  return orc_basic_keyed(fid, dim, seed, (uint32_t)fid << 8, t->s, t->c, t->rotated, 0);
}

/* Basic formula `base` under a caller-chosen transform; `id` keys the random streams. */
orc_problem *orc_problem_custom_basic(int id, int base, int dim, uint64_t seed, double s, double c, int rotated) {
  return orc_basic_keyed(base, dim, seed, (uint32_t)id << 8, s, c, rotated, 0);
}

/* Sec. 5: y = x - o; S permutes y; group i takes the next n_i entries, n_i = ceil(p_i D) for
 * i < N and the remainder for the last; F = sum_i G_i(R_i z^i) + f_opt.  Reading: each G_i
 * applies its own scale and offset, g_i(R_i (s_i z^i) + c_i), at dimension n_i. */
static orc_problem *orc_hybrid_keyed(int dim, uint64_t seed, uint32_t key, int ng, const int *bases,
                                     const double *p) {
  if (ng < 1 || ng > ORC_MAXC || dim < 2) return NULL;
  int sizes[ORC_MAXC];
  int used = 0;
  for (int i = 0; i + 1 < ng; ++i) {
    sizes[i] = (int)ceil(p[i] * (double)dim);
    used += sizes[i];
  }
  sizes[ng - 1] = dim - used;
  /* a group needs one variable, two for the formulas that divide by (n - 1): the elliptic and
     different-powers exponents (i-1)/(n-1) and Schaffer's F7 mean over n-1 pairs */
  for (int i = 0; i < ng; ++i) {
    if (bases[i] < 0 || bases[i] > 22 || sizes[i] < 1) return NULL;
    if (sizes[i] < 2 && (bases[i] == 2 || bases[i] == 5 || bases[i] == 12)) return NULL;
  }
  orc_problem *h = orc_alloc(ORC_HYBRID, dim);
  h->ngroups = ng;
  h->o = (double *)malloc(sizeof(double) * (size_t)dim);
  orc_make_shift(seed, dim, key, h->o);
  h->perm = (int *)malloc(sizeof(int) * (size_t)dim);
  orc_make_perm(seed, dim, key, h->perm);
  orc_rng g;
  orc_rng_open(&g, seed, dim, key, 2);
  for (int i = 0; i < ng; ++i) {
    h->gbase[i] = bases[i];
    h->gsize[i] = sizes[i];
    h->gR[i] = (double *)malloc(sizeof(double) * (size_t)sizes[i] * (size_t)sizes[i]);
    orc_draw_block(&g, sizes[i], h->gR[i]);
  }
  return h;
}

orc_problem *orc_problem_hybrid(int id, int dim, uint64_t seed, int ng, const int *bases, const double *p) {
  return orc_hybrid_keyed(dim, seed, (uint32_t)id << 8, ng, bases, p);
}

/* Sec. 6: F = sum_i omega_i (lambda_i G_i(x) + bias_i) + f_opt, where component i is a
 * basic function with its own optimum and rotation. */
orc_problem *orc_problem_composition(int id, int dim, uint64_t seed, int nc, const int *bases, const double *sigma,
                                     const double *lambda, const double *bias) {
  if (nc < 1 || nc > ORC_MAXC || dim < 2) return NULL;
  orc_problem *q = orc_alloc(ORC_COMPOSITION, dim);
  q->ncomp = nc;
  for (int i = 0; i < nc; ++i) {
    if (bases[i] < 0 || bases[i] > 22) {
      orc_problem_free(q);
      return NULL;
    }
    const orc_xform_t *t = &ORC_XF[bases[i]];
    q->comp[i] = orc_basic_keyed(bases[i], dim, seed, ((uint32_t)id << 8) | (uint32_t)i, t->s, t->c, t->rotated, 0);
    q->sigma[i] = sigma[i];
    q->lambda[i] = lambda[i];
    q->cbias[i] = bias[i];
  }
  return q;
}

/* The paper's fixed hybrid (Secs. 5.1-5.6) and composition (Secs. 6.1-6.8) tables.
 * Parity unpinned against the original data; see the readings in the design notes. */
static const int ORC_HY_N[6] = {3, 3, 4, 4, 5, 5};
static const double ORC_HY_P[6][5] = {{0.3, 0.3, 0.4}, {0.3, 0.3, 0.4}, {0.2, 0.2, 0.3, 0.3},
                                      {0.2, 0.2, 0.3, 0.3}, {0.1, 0.2, 0.2, 0.2, 0.3}, {0.1, 0.2, 0.2, 0.2, 0.3}};
static const int ORC_HY_G[6][5] = {{15, 10, 2}, {4, 21, 10}, {9, 8, 14, 22}, {21, 3, 13, 10}, {22, 21, 14, 15, 2},
                                   {17, 20, 13, 15, 19}};

orc_problem *orc_problem_paper_hybrid(int fid, int dim, uint64_t seed) {
  if (fid < 23 || fid > 28) return NULL;
  int h = fid - 23;
  return orc_hybrid_keyed(dim, seed, (uint32_t)fid << 8, ORC_HY_N[h], ORC_HY_G[h], ORC_HY_P[h]);
}

static const int ORC_CO_N[8] = {5, 3, 3, 5, 5, 5, 3, 3};
static const double ORC_CO_SIG[8][5] = {{10, 20, 30, 40, 50}, {15, 15, 15}, {20, 50, 40}, {20, 15, 10, 10, 40},
                                        {15, 15, 15, 15, 15}, {10, 20, 30, 40, 50}, {10, 30, 50}, {10, 30, 50}};
static const double ORC_CO_LAM[8][5] = {{1e-10, 1e-6, 1e-26, 1e-6, 1e-6}, {1, 1, 1}, {0.25, 1, 1e-7},
                                        {2.5e-2, 0.1, 1e-8, 0.25, 1}, {10, 10, 2.5, 2.5, 1e-6},
                                        {2.5, 10, 2.5, 5e-4, 1e-6}, {1, 1, 1}, {1, 1, 1}};
/* component ids; >= 23 means the paper hybrid of that id */
static const int ORC_CO_G[8][5] = {{14, 2, 4, 3, 2}, {15, 11, 21}, {16, 11, 2}, {16, 20, 2, 8, 9},
                                   {21, 11, 16, 8, 2}, {13, 20, 16, 22, 2}, {23, 24, 25}, {26, 27, 28}};

orc_problem *orc_problem_paper_composition(int fid, int dim, uint64_t seed) {
  if (fid < 29 || fid > 36) return NULL;
  int c = fid - 29;
  orc_problem *q = orc_alloc(ORC_COMPOSITION, dim);
  q->ncomp = ORC_CO_N[c];
  for (int i = 0; i < q->ncomp; ++i) {
    int g = ORC_CO_G[c][i];
    uint32_t key = ((uint32_t)fid << 8) | (uint32_t)i;
    if (g >= 23) {
      int h = g - 23;
      q->comp[i] = orc_hybrid_keyed(dim, seed, key, ORC_HY_N[h], ORC_HY_G[h], ORC_HY_P[h]);
      /* the trap of Sec. 6: the third component's optimum sits at the origin */
      if (q->comp[i] && i == 2) memset(q->comp[i]->o, 0, sizeof(double) * (size_t)dim);
    } else {
      const orc_xform_t *t = &ORC_XF[g];
      q->comp[i] = orc_basic_keyed(g, dim, seed, key, t->s, t->c, t->rotated, i == 2);
    }
    if (!q->comp[i]) {
      orc_problem_free(q);
      return NULL;
    }
    q->sigma[i] = ORC_CO_SIG[c][i];
    q->lambda[i] = ORC_CO_LAM[c][i];
    q->cbias[i] = 100.0 * (double)i;
  }
  return q;
}

/* Any Tab. 1 id 0..36. */
orc_problem *orc_problem_fid(int fid, int dim, uint64_t seed) {
  if (fid >= 0 && fid <= 22) return orc_problem_basic(fid, dim, seed);
  if (fid >= 23 && fid <= 28) return dim >= 10 ? orc_problem_paper_hybrid(fid, dim, seed) : NULL;
  if (fid >= 29 && fid <= 36) {
    if ((fid == 35 || fid == 36) && dim < 10) return NULL;
    return orc_problem_paper_composition(fid, dim, seed);
  }
  return NULL;
}

void orc_problem_free(orc_problem *p) {
  if (!p) return;
  free(p->o);
  free(p->R);
  free(p->perm);
  for (int i = 0; i < ORC_MAXC; ++i) {
    free(p->gR[i]);
    orc_problem_free(p->comp[i]);
  }
  free(p);
}

/* ------------------------------------------------------------------------------------------
 * Evaluation
 * ---------------------------------------------------------------------------------------- */

/* z = R (s (x - o)) + c for a basic problem; `y` is scratch of length D. */
static void orc_basic_transform(const orc_problem *p, const double *x, double *y, double *z) {
  int D = p->dim;
  for (int j = 0; j < D; ++j) y[j] = p->s * (x[j] - p->o[j]);
  for (int i = 0; i < D; ++i) {
    double acc;
    if (p->R) {
      acc = 0.0;
      for (int j = 0; j < D; ++j) acc += p->R[(size_t)i * D + j] * y[j];
    } else {
      acc = y[i];
    }
    z[i] = acc + p->c;
  }
}

/* value without f_opt; scratch needs 3*D doubles */
static double orc_value(const orc_problem *p, const double *x, double *scratch) {
  int D = p->dim;
  if (p->kind == ORC_BASIC) {
    double *y = scratch, *z = scratch + D;
    orc_basic_transform(p, x, y, z);
    return ORC_G[p->base](D, z);
  }
  if (p->kind == ORC_HYBRID) {
    double *y = scratch, *v = scratch + D, *z = scratch + 2 * D;
    for (int j = 0; j < D; ++j) y[j] = x[j] - p->o[j];
    double F = 0.0;
    int off = 0;
    for (int g = 0; g < p->ngroups; ++g) {
      int n = p->gsize[g];
      const orc_xform_t *t = &ORC_XF[p->gbase[g]];
      for (int a = 0; a < n; ++a) v[a] = t->s * y[p->perm[off + a]];
      for (int a = 0; a < n; ++a) {
        double acc = 0.0;
        for (int b = 0; b < n; ++b) acc += p->gR[g][a * n + b] * v[b];
        z[a] = acc + t->c;
      }
      F += ORC_G[p->gbase[g]](n, z);
      off += n;
    }
    return F;
  }
  /* composition, Eq. (composition) and Eq. (weight) */
  double w[ORC_MAXC], G[ORC_MAXC];
  int nzero = 0;
  for (int i = 0; i < p->ncomp; ++i) {
    const orc_problem *c = p->comp[i];
    double d2 = 0.0;
    for (int j = 0; j < D; ++j) d2 += (x[j] - c->o[j]) * (x[j] - c->o[j]);
    G[i] = orc_value(c, x, scratch);
    if (d2 == 0.0) {
      w[i] = -1.0; /* marks x == x_opt,i: the weights become one-hot there */
      ++nzero;
    } else {
      w[i] = (1.0 / sqrt(d2)) * exp(-d2 / (2.0 * (double)D * p->sigma[i] * p->sigma[i]));
    }
  }
  double sw = 0.0;
  if (nzero > 0) {
    for (int i = 0; i < p->ncomp; ++i) w[i] = (w[i] == -1.0) ? 1.0 : 0.0;
  }
  for (int i = 0; i < p->ncomp; ++i) sw += w[i];
  double F = 0.0;
  for (int i = 0; i < p->ncomp; ++i) F += (w[i] / sw) * (p->lambda[i] * G[i] + p->cbias[i]);
  return F;
}

/* f for n row-major candidate vectors; nthreads <= 1 runs single-threaded. */
int orc_evaluate(const orc_problem *p, const double *x, long n, double *f, int nthreads) {
  if (!p) return -1;
  int D = p->dim;
#ifdef _OPENMP
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
#endif
  {
    double *scratch = (double *)malloc(sizeof(double) * 3 * (size_t)D);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
    for (long r = 0; r < n; ++r) f[r] = orc_value(p, x + (size_t)r * D, scratch) + p->fopt;
    free(scratch);
  }
  return 0;
}

/* ------------------------------------------------------------------------------------------
 * Accessors for the self-tests
 * ---------------------------------------------------------------------------------------- */
int orc_problem_dim(const orc_problem *p) { return p ? p->dim : -1; }
int orc_problem_kind(const orc_problem *p) { return p ? p->kind : -1; }
int orc_problem_ncomp(const orc_problem *p) {
  if (!p) return -1;
  return p->kind == ORC_COMPOSITION ? p->ncomp : (p->kind == ORC_HYBRID ? p->ngroups : 1);
}

/* shift vector of the problem (component `i` for compositions) */
int orc_problem_shift(const orc_problem *p, int i, double *o) {
  if (!p) return -1;
  const orc_problem *q = p->kind == ORC_COMPOSITION ? (i >= 0 && i < p->ncomp ? p->comp[i] : NULL) : p;
  if (!q) return -1;
  memcpy(o, q->o, sizeof(double) * (size_t)q->dim);
  return 0;
}

/* dense rotation of a basic problem (component `i` for compositions); identity if unrotated */
int orc_problem_rotation(const orc_problem *p, int i, double *R) {
  if (!p) return -1;
  const orc_problem *q = p->kind == ORC_COMPOSITION ? (i >= 0 && i < p->ncomp ? p->comp[i] : NULL) : p;
  if (!q || q->kind != ORC_BASIC) return -1;
  int D = q->dim;
  if (q->R)
    memcpy(R, q->R, sizeof(double) * (size_t)D * (size_t)D);
  else {
    memset(R, 0, sizeof(double) * (size_t)D * (size_t)D);
    for (int j = 0; j < D; ++j) R[(size_t)j * D + j] = 1.0;
  }
  return 0;
}

/* hybrid: permutation S, group sizes and the group rotations packed one after another */
int orc_problem_hybrid_parts(const orc_problem *p, int *perm, int *sizes, double *blocks) {
  if (!p || p->kind != ORC_HYBRID) return -1;
  memcpy(perm, p->perm, sizeof(int) * (size_t)p->dim);
  size_t off = 0;
  for (int g = 0; g < p->ngroups; ++g) {
    sizes[g] = p->gsize[g];
    size_t nn = (size_t)p->gsize[g] * (size_t)p->gsize[g];
    memcpy(blocks + off, p->gR[g], sizeof(double) * nn);
    off += nn;
  }
  return p->ngroups;
}

/* z of a basic problem at one point (transform only, Sec. 1.2 / each "where" clause) */
int orc_problem_transform(const orc_problem *p, const double *x, double *z) {
  if (!p || p->kind != ORC_BASIC) return -1;
  double *y = (double *)malloc(sizeof(double) * (size_t)p->dim);
  orc_basic_transform(p, x, y, z);
  free(y);
  return 0;
}

/* g(z) of Tab. 1 formula `fid` (0..22) on an arbitrary z, without bias */
double orc_g(int fid, int n, const double *z) {
  if (fid < 0 || fid > 22 || n < 1) return NAN;
  return ORC_G[fid](n, z);
}

/* raw generator streams, for pinning the generator itself */
void orc_stream_u64(uint64_t seed, int dim, uint32_t key, uint32_t purpose, long n, uint64_t *out) {
  orc_rng g;
  orc_rng_open(&g, seed, dim, key, purpose);
  for (long i = 0; i < n; ++i) out[i] = orc_next(&g);
}
void orc_stream_normal(uint64_t seed, int dim, uint32_t key, uint32_t purpose, long n, double *out) {
  orc_rng g;
  orc_rng_open(&g, seed, dim, key, purpose);
  for (long i = 0; i < n; ++i) out[i] = orc_normal(&g);
}
uint64_t orc_splitmix64_from_state(uint64_t state, long k) {
  uint64_t v = 0;
  for (long i = 0; i <= k; ++i) {
    state += 0x9E3779B97F4A7C15ULL;
    v = orc_mix64(state);
  }
  return v;
}
/* CGS2 on a caller matrix, to pin it against a library QR */
void orc_orthonormalise(int n, double *A) { orc_cgs2(n, A); }

int orc_num_threads_available(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------------------------
 * The transcribed parameter tables and the parameters of constructed problems, so that tests
 * can compare both with the values the paper prints (Secs. 3-6).
 * ---------------------------------------------------------------------------------------- */

/* scale, offset and rotation flag of Tab. 1 function fid (0..22), Secs. 3-4 */
int orc_table_xform(int fid, double *s, double *c, int *rotated) {
  if (fid < 0 || fid > 22) return -1;
  *s = ORC_XF[fid].s;
  *c = ORC_XF[fid].c;
  *rotated = ORC_XF[fid].rotated;
  return 0;
}

/* Secs. 5.1-5.6: proportions p and component ids G of hybrid fid (23..28); returns N */
int orc_table_hybrid(int fid, double *p, int *g) {
  if (fid < 23 || fid > 28) return -1;
  int h = fid - 23;
  for (int i = 0; i < ORC_HY_N[h]; ++i) {
    p[i] = ORC_HY_P[h][i];
    g[i] = ORC_HY_G[h][i];
  }
  return ORC_HY_N[h];
}

/* Secs. 6.1-6.8: sigma, lambda and component ids of composition fid (29..36); returns N */
int orc_table_composition(int fid, double *sigma, double *lambda, int *g) {
  if (fid < 29 || fid > 36) return -1;
  int c = fid - 29;
  for (int i = 0; i < ORC_CO_N[c]; ++i) {
    sigma[i] = ORC_CO_SIG[c][i];
    lambda[i] = ORC_CO_LAM[c][i];
    g[i] = ORC_CO_G[c][i];
  }
  return ORC_CO_N[c];
}

/* formula id, scale, offset and rotation flag a basic problem was built with */
int orc_problem_basic_params(const orc_problem *p, int *base, double *s, double *c, int *rotated) {
  if (!p || p->kind != ORC_BASIC) return -1;
  *base = p->base;
  *s = p->s;
  *c = p->c;
  *rotated = p->R != NULL;
  return 0;
}

/* formula ids of the groups of a hybrid problem; returns the group count */
int orc_problem_group_bases(const orc_problem *p, int *bases) {
  if (!p || p->kind != ORC_HYBRID) return -1;
  for (int g = 0; g < p->ngroups; ++g) bases[g] = p->gbase[g];
  return p->ngroups;
}

/* sigma_i, lambda_i and bias_i a composition was built with; returns the component count */
int orc_problem_blend_params(const orc_problem *p, double *sigma, double *lambda, double *bias) {
  if (!p || p->kind != ORC_COMPOSITION) return -1;
  for (int i = 0; i < p->ncomp; ++i) {
    sigma[i] = p->sigma[i];
    lambda[i] = p->lambda[i];
    bias[i] = p->cbias[i];
  }
  return p->ncomp;
}

/* component i of a composition (owned by the composition, valid while it lives) */
const orc_problem *orc_problem_component(const orc_problem *p, int i) {
  if (!p || p->kind != ORC_COMPOSITION || i < 0 || i >= p->ncomp) return NULL;
  return p->comp[i];
}

/* ------------------------------------------------------------------------------------------
 * Differential evolution (DE/rand/1/bin) with the FP64 formulas above: the optimiser-in-the-loop
 * use the paper motivates (Sec. 1) and measures with 50 concurrent evaluations (Sec. 2), as a
 * reference for the GPU optimiser.  Draws are counter based, SplitMix64's output for the state
 * seed + (k + 1) * 0x9E3779B97F4A7C15, draw k = (g * np + i) * (D + 4) + slot for individual i
 * of generation g: slots 0-2 choose r1, r2, r3 among the indices not yet taken (i first), as
 * the v-th remaining index in increasing order with v = draw mod count; slot 3 the forced
 * position draw mod D; slot 4 + j the crossover uniform (draw >> 11) 2^-53 of variable j.
 * Trial: fma(F, x_r2 - x_r3, x_r1) clamped to [-100, 100] where the uniform is below CR or at the
 * forced position, the target's value elsewhere; a trial whose value is not larger replaces
 * its target.  pop (np x D) and fit (np) are updated in place over `generations` generations
 * starting at generation gen0.  Returns the smallest |f_trial - f_target| / max(1, |f_target|)
 * met in a selection (how close the closest decision was).
 * ---------------------------------------------------------------------------------------- */
static uint64_t orc_counter_draw(uint64_t seed, uint64_t k) {
  return orc_mix64(seed + (k + 1u) * 0x9E3779B97F4A7C15ULL);
}

double orc_de_run(const orc_problem *p, int np, double F, double CR, uint64_t seed, uint64_t gen0, int generations,
                  double *pop, double *fit) {
  int D = p->dim;
  double *trial = (double *)malloc(sizeof(double) * (size_t)np * (size_t)D);
  double *ft = (double *)malloc(sizeof(double) * (size_t)np);
  int *avail = (int *)malloc(sizeof(int) * (size_t)np);
  double margin = INFINITY;
  for (int gi = 0; gi < generations; ++gi) {
    uint64_t g = gen0 + (uint64_t)gi;
    for (int i = 0; i < np; ++i) {
      uint64_t base = ((uint64_t)g * (uint64_t)np + (uint64_t)i) * (uint64_t)(D + 4);
      /* indices still allowed, in increasing order; take i out first */
      int navail = 0;
      for (int a = 0; a < np; ++a)
        if (a != i) avail[navail++] = a;
      int r[3];
      for (int t = 0; t < 3; ++t) {
        int v = (int)(orc_counter_draw(seed, base + (uint64_t)t) % (uint64_t)navail);
        r[t] = avail[v];
        for (int a = v; a + 1 < navail; ++a) avail[a] = avail[a + 1];
        --navail;
      }
      int jr = (int)(orc_counter_draw(seed, base + 3) % (uint64_t)D);
      for (int j = 0; j < D; ++j) {
        double u = (double)(orc_counter_draw(seed, base + 4 + (uint64_t)j) >> 11) * 0x1.0p-53;
        double v = pop[(size_t)i * D + j];
        if (u < CR || j == jr) {
          v = fma(F, pop[(size_t)r[1] * D + j] - pop[(size_t)r[2] * D + j], pop[(size_t)r[0] * D + j]);
          if (v < -100.0) v = -100.0;
          if (v > 100.0) v = 100.0;
        }
        trial[(size_t)i * D + j] = v;
      }
    }
    orc_evaluate(p, trial, np, ft, 1);
    for (int i = 0; i < np; ++i) {
      double m = fabs(ft[i] - fit[i]) / fmax(1.0, fabs(fit[i]));
      if (m < margin) margin = m;
      if (ft[i] <= fit[i]) {
        memcpy(pop + (size_t)i * D, trial + (size_t)i * D, sizeof(double) * (size_t)D);
        fit[i] = ft[i];
      }
    }
  }
  free(trial);
  free(ft);
  free(avail);
  return margin;
}
