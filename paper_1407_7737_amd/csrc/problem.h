// problem.h -- host-side problem definitions of the cuROB suite (arXiv 1407.7737) and the
// device tables the evaluation kernels read.  Host code only (no device code in here).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace curob {

// Formula families the kernels implement; several Tab. 1 ids share one family and differ only
// in a per-index coefficient (e.g. sphere/ellipsoid/elliptic/discus/cigar are all sum w_i z_i^2).
enum Kind : int {
  K_WSPHERE = 0,   // sum w_i z_i^2                      (ids 0-4, Secs. 3.1-3.5)
  K_POWERS,        // sqrt(sum |z_i|^e_i)                (id 5, Sec. 3.6)
  K_SHARPV,        // z_1^2 + 100 sqrt(sum_{i>1} z_i^2)  (id 6, Sec. 3.7)
  K_STEP,          // sum floor(z_i + 1/2)^2             (id 7, Sec. 4.1)
  K_WEIERSTRASS,   // (id 8, Sec. 4.2)
  K_GRIEWANK,      // (id 9, Sec. 4.3)
  K_RASTRIGIN,     // (ids 10, 11, Secs. 4.4-4.5)
  K_F7,            // Schaffer F7, neighbour pairs       (id 12, Sec. 4.6)
  K_GRIEROSEN,     // neighbour pairs with wrap          (id 13, Sec. 4.7)
  K_ROSENBROCK,    // neighbour pairs                    (id 14, Sec. 4.8)
  K_SCHWEFEL,      // (ids 15, 16, Secs. 4.9-4.10)
  K_KATSUURA,      // (id 17, Sec. 4.11)
  K_LUNACEK,       // (id 18, Sec. 4.12)
  K_ACKLEY,        // (id 19, Sec. 4.13)
  K_HAPPYCAT,      // (id 20, Sec. 4.14)
  K_HGBAT,         // (id 21, Sec. 4.15)
  K_F6,            // expanded Schaffer F6, pairs + wrap (id 22, Sec. 4.16)
  K_COUNT
};

// Constant added to z before a family's terms, folded into the c' tables (constexpr: usable in
// device code too): HappyCat and HGBat (Secs. 4.14-4.15) take w = z + 1, since their optimum sits
// at z = -1 and terms written in w keep their precision as w -> 0, where terms written in z ~ -1
// cancel.  (Schwefel's g1 takes z + 420.9687462275036 too, but adds it in the formula, which
// needs z itself near the optimum.)
constexpr double kind_zshift(int kind) { return (kind == K_HAPPYCAT || kind == K_HGBAT) ? 1.0 : 0.0; }

// Schwefel's g1 argument offset w* = 420.9687462275036 (Sec. 4.9).
constexpr double kSchwefelW = 420.9687462275036;

// Schwefel's constant 418.9829, kept as printed (Sec. 4.9).
constexpr double kSchwefelC = 418.9829;

// Transform and formula of one Tab. 1 basic function.
struct FnSpec {
  int kind;
  double s;      // scale inside the rotation
  double c;      // offset added after the rotation
  bool rotated;
};
const FnSpec &fn_spec(int base);  // base in 0..22
bool kind_is_pairwise(int kind);
bool kind_pair_wraps(int kind);
int min_dimension(int base);  // smallest dimension the formula is defined for
// FP32 split mode: formulas (at the dimension n the formula sees) that get the six-product rotation
bool needs_six_products(int base, int n);

// SplitMix64 stream (Steele, Lea & Flood 2014) with Marsaglia-polar normals.
class Rng {
 public:
  // independent stream per (seed, dimension, problem key, purpose); purpose 0 = shift,
  // 1 = permutation, 2 = rotation entries
  Rng(uint64_t seed, int dim, uint32_t key, uint32_t purpose);
  uint64_t next_u64();
  double uniform();  // [0,1), 53 random bits
  double normal();

 private:
  uint64_t state_;
  bool have_spare_ = false;
  double spare_ = 0.0;
};

// Replaces the n x n row-major A by the orthonormal factor Q of A = QR with diag(R) > 0,
// computed with Householder reflections.
void orthonormal_factor(int n, std::vector<double> &A);

// One formula segment over a range of the packed (group-ordered) variable space.
struct Segment {
  int base;   // Tab. 1 id 0..22
  int off;    // first packed position
  int n;      // length (the dimension the formula sees)
  double s, c;
};

struct Problem {
  enum { BASIC = 0, HYBRID = 1, COMPOSITION = 2 };
  int type = BASIC;
  int dim = 0;
  double fopt = 100.0;  // Tab. 1: f_opt = 100 for every function
  // basic and hybrid
  std::vector<double> o;           // shift, original variable order
  std::vector<int> orig;           // packed position -> original variable
  bool rotated = false;
  std::vector<int> blk_off, blk_n; // rotation blocks in packed space
  std::vector<std::vector<double>> Q;  // one n x n block each
  std::vector<Segment> segs;       // basic: one segment over all D; hybrid: one per group
  bool index_by_original = true;   // basic: formula index = original variable; hybrid: position in group
  // composition
  std::vector<Problem> comps;
  std::vector<double> sigma, lambda, cbias;
};

Problem make_basic(int base, int dim, uint64_t seed, uint32_t key, double s, double c, bool rotated,
                   bool origin_optimum);
Problem make_tab1_basic(int fid, int dim, uint64_t seed);
// ngroups groups, sizes from proportions p (Eq. (numbers)); throws std::invalid_argument
Problem make_hybrid(int dim, uint64_t seed, uint32_t key, int ngroups, const int *bases, const double *p);
Problem make_composition(int dim, uint64_t seed, uint32_t key, int ncomp, const int *bases, const double *sigma,
                         const double *lambda, const double *bias);
Problem make_tab1(int fid, int dim, uint64_t seed);  // any id 0..36

// Split mode on a whole problem: six products when any of its formulas needs them.
bool problem_needs_six(const Problem &p);

// Dense D x D rotation of a basic problem in original variable order (identity if unrotated).
std::vector<double> dense_rotation(const Problem &p);

// Per-position coefficient of a formula: w_i for the weighted-sphere family, exponents for
// powers, 1/sqrt(i) for Griewank, the index for Katsuura, a first-element flag for sharp valley.
double formula_coef(int base, int i, int n);

}  // namespace curob
