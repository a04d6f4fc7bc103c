// problem.cpp -- problem generation for the cuROB suite (General Setup, Sec. 1.2; hybrid
// functions, Sec. 5; composition functions, Sec. 6).  Host code, FP64.
#include "problem.h"

#include <cmath>
#include <stdexcept>

namespace curob {

namespace {

const FnSpec kSpecs[23] = {
    {K_WSPHERE, 1.0, 0.0, true},       // 0 sphere (Sec. 3.1)
    {K_WSPHERE, 1.0, 0.0, true},       // 1 ellipsoid (Sec. 3.2)
    {K_WSPHERE, 1.0, 0.0, true},       // 2 high-conditioned elliptic (Sec. 3.3)
    {K_WSPHERE, 1.0, 0.0, true},       // 3 discus (Sec. 3.4)
    {K_WSPHERE, 1.0, 0.0, true},       // 4 bent cigar (Sec. 3.5)
    {K_POWERS, 0.01, 0.0, true},       // 5 different powers (Sec. 3.6)
    {K_SHARPV, 1.0, 0.0, true},        // 6 sharp valley (Sec. 3.7)
    {K_STEP, 1.0, 0.0, true},          // 7 step (Sec. 4.1)
    {K_WEIERSTRASS, 0.005, 0.0, true}, // 8 Weierstrass (Sec. 4.2)
    {K_GRIEWANK, 6.0, 0.0, true},      // 9 Griewank (Sec. 4.3)
    {K_RASTRIGIN, 0.0512, 0.0, false}, // 10 shifted Rastrigin (Sec. 4.4)
    {K_RASTRIGIN, 0.0512, 0.0, true},  // 11 rotated Rastrigin (Sec. 4.5)
    {K_F7, 1.0, 0.0, true},            // 12 Schaffer F7 (Sec. 4.6)
    {K_GRIEROSEN, 0.05, 1.0, true},    // 13 expanded Griewank plus Rosenbrock (Sec. 4.7)
    {K_ROSENBROCK, 0.02048, 1.0, true},// 14 Rosenbrock (Sec. 4.8)
    {K_SCHWEFEL, 10.0, 0.0, false},    // 15 modified Schwefel (Sec. 4.9)
    {K_SCHWEFEL, 10.0, 0.0, true},     // 16 rotated modified Schwefel (Sec. 4.10)
    {K_KATSUURA, 0.05, 0.0, true},     // 17 Katsuura (Sec. 4.11)
    {K_LUNACEK, 0.1, 2.5, true},       // 18 Lunacek bi-Rastrigin (Sec. 4.12), offset outside R
    {K_ACKLEY, 1.0, 0.0, true},        // 19 Ackley (Sec. 4.13)
    {K_HAPPYCAT, 0.05, -1.0, true},    // 20 HappyCat (Sec. 4.14)
    {K_HGBAT, 0.05, -1.0, true},       // 21 HGBat (Sec. 4.15)
    {K_F6, 1.0, 0.0, true},            // 22 expanded Schaffer F6 (Sec. 4.16)
};

inline uint64_t finalize64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Fisher-Yates shuffle of 0..D-1 from the permutation stream.
std::vector<int> random_permutation(uint64_t seed, int dim, uint32_t key) {
  Rng g(seed, dim, key, 1);
  std::vector<int> perm(dim);
  for (int j = 0; j < dim; ++j) perm[j] = j;
  for (int i = dim - 1; i >= 1; --i) {
    int j = static_cast<int>(g.next_u64() % static_cast<uint64_t>(i + 1));
    std::swap(perm[i], perm[j]);
  }
  return perm;
}

std::vector<double> random_shift(uint64_t seed, int dim, uint32_t key) {
  Rng g(seed, dim, key, 0);
  std::vector<double> o(dim);
  for (int j = 0; j < dim; ++j) o[j] = -70.0 + 140.0 * g.uniform();  // x_opt in [-70,70]^D
  return o;
}

std::vector<double> random_block(Rng &g, int n) {
  std::vector<double> A(static_cast<size_t>(n) * n);
  for (auto &v : A) v = g.normal();
  orthonormal_factor(n, A);
  return A;
}

}  // namespace

const FnSpec &fn_spec(int base) { return kSpecs[base]; }

bool kind_is_pairwise(int kind) {
  return kind == K_F7 || kind == K_GRIEROSEN || kind == K_ROSENBROCK || kind == K_F6;
}
bool kind_pair_wraps(int kind) { return kind == K_GRIEROSEN || kind == K_F6; }

// Formulas whose FP32 value amplifies a relative error of z far beyond its own size: the
// 1e6-weighted single components of elliptic and discus, the plateaus of step, the 3^k
// and 2^j frequencies of Weierstrass and Katsuura, the phases 50 w^0.2 (Schaffer F7) and
// g2(z_i, z_{i+1}) (Griewank-Rosenbrock), and the jumps of the rotated Schwefel g1 at
// |w| = 1000, 1500, ...  For these the split rotation uses six BF16 products.  Rosenbrock's
// pair term amplifies the z error by up to |400 z_i (z_i^2 - z_{i+1})| / f; the three-product
// rotation (z error ~ 2^-16 |z|) meets the FP32 bar once several pairs average their errors,
// but not with one or a few pairs, so low dimensions get six products as well.  The same
// holds for the elliptic sum: with few variables one 1e6-weighted z carries f, and its
// relative error is the rotation's; from 50 variables on the measured three-product error
// stays below a fifth of the FP32 bar (a tenth at 100 and 128).
bool needs_six_products(int base, int n) {
  switch (base) {
    case 3: case 7: case 8: case 12: case 13: case 16: case 17: return true;
    case 2: return n < 50;
    case 4: return n < 10;  // bent cigar: with few variables one or two 1e6-weighted z carry f
    case 14: return n < 10;
    default: return false;
  }
}

bool problem_needs_six(const Problem &p) {
  for (const Segment &sg : p.segs)
    if (needs_six_products(sg.base, sg.n)) return true;
  for (const Problem &c : p.comps)
    if (problem_needs_six(c)) return true;
  return false;
}

// The elliptic and powers exponents (i-1)/(n-1) and the F7 mean over n-1 pairs need n >= 2.
int min_dimension(int base) { return (base == 2 || base == 5 || base == 12) ? 2 : 1; }

Rng::Rng(uint64_t seed, int dim, uint32_t key, uint32_t purpose) {
  uint64_t tag = (static_cast<uint64_t>(key) << 32) ^ (static_cast<uint64_t>(purpose) << 24) ^
                 static_cast<uint64_t>(static_cast<uint32_t>(dim));
  state_ = finalize64(seed ^ finalize64(tag));
}

uint64_t Rng::next_u64() {
  state_ += 0x9E3779B97F4A7C15ULL;
  return finalize64(state_);
}

double Rng::uniform() { return static_cast<double>(next_u64() >> 11) * 0x1.0p-53; }

double Rng::normal() {
  if (have_spare_) {
    have_spare_ = false;
    return spare_;
  }
  double u, v, r2;
  do {
    u = 2.0 * uniform() - 1.0;
    v = 2.0 * uniform() - 1.0;
    r2 = u * u + v * v;
  } while (r2 >= 1.0 || r2 == 0.0);
  double m = std::sqrt(-2.0 * std::log(r2) / r2);
  spare_ = v * m;
  have_spare_ = true;
  return u * m;
}

// Householder QR: reflect column j below the diagonal to a multiple of e_j, accumulate
// Q = H_0 H_1 ... H_{n-1}, then flip column signs so that diag(R) > 0.  The orthonormal
// factor with positive diagonal is unique, which is what Sec. 1.2's Gram-Schmidt produces.
void orthonormal_factor(int n, std::vector<double> &A) {
  std::vector<double> R(A);  // working copy, becomes R
  std::vector<std::vector<double>> vs(n);
  std::vector<double> betas(n, 0.0);
  for (int j = 0; j < n; ++j) {
    double norm2 = 0.0;
    for (int r = j; r < n; ++r) norm2 += R[r * n + j] * R[r * n + j];
    double alpha = std::sqrt(norm2);
    double x0 = R[j * n + j];
    std::vector<double> v(n - j);
    for (int r = j; r < n; ++r) v[r - j] = R[r * n + j];
    v[0] = x0 >= 0.0 ? x0 + alpha : x0 - alpha;
    double vnorm2 = 0.0;
    for (double t : v) vnorm2 += t * t;
    double beta = vnorm2 > 0.0 ? 2.0 / vnorm2 : 0.0;
    for (int c = j; c < n; ++c) {
      double d = 0.0;
      for (int r = j; r < n; ++r) d += v[r - j] * R[r * n + c];
      d *= beta;
      for (int r = j; r < n; ++r) R[r * n + c] -= d * v[r - j];
    }
    vs[j] = std::move(v);
    betas[j] = beta;
  }
  // Q = H_0 ... H_{n-1} applied to the identity, right to left
  std::vector<double> Qm(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) Qm[i * n + i] = 1.0;
  for (int j = n - 1; j >= 0; --j) {
    const std::vector<double> &v = vs[j];
    for (int c = 0; c < n; ++c) {
      double d = 0.0;
      for (int r = j; r < n; ++r) d += v[r - j] * Qm[r * n + c];
      d *= betas[j];
      for (int r = j; r < n; ++r) Qm[r * n + c] -= d * v[r - j];
    }
  }
  for (int c = 0; c < n; ++c) {
    if (R[c * n + c] < 0.0)
      for (int r = 0; r < n; ++r) Qm[r * n + c] = -Qm[r * n + c];
  }
  A.swap(Qm);
}

Problem make_basic(int base, int dim, uint64_t seed, uint32_t key, double s, double c, bool rotated,
                   bool origin_optimum) {
  if (base < 0 || base > 22) throw std::invalid_argument("base function id must be in 0..22");
  if (dim < 2) throw std::invalid_argument("dimension must be at least 2");
  Problem p;
  p.type = Problem::BASIC;
  p.dim = dim;
  p.o = origin_optimum ? std::vector<double>(dim, 0.0) : random_shift(seed, dim, key);
  p.rotated = rotated;
  p.index_by_original = true;
  if (rotated) {
    // three (almost) equal random groups, each rotated by its own orthonormal block (Sec. 1.2)
    p.orig = random_permutation(seed, dim, key);
    Rng g(seed, dim, key, 2);
    int off = 0;
    for (int k = 0; k < 3; ++k) {
      int nk = dim / 3 + (k < dim % 3 ? 1 : 0);
      if (nk == 0) continue;
      p.blk_off.push_back(off);
      p.blk_n.push_back(nk);
      p.Q.push_back(random_block(g, nk));
      off += nk;
    }
  } else {
    p.orig.resize(dim);
    for (int j = 0; j < dim; ++j) p.orig[j] = j;
  }
  p.segs.push_back(Segment{base, 0, dim, s, c});
  return p;
}

Problem make_tab1_basic(int fid, int dim, uint64_t seed) {
  const FnSpec &t = fn_spec(fid);
  return make_basic(fid, dim, seed, static_cast<uint32_t>(fid) << 8, t.s, t.c, t.rotated, false);
}

Problem make_hybrid(int dim, uint64_t seed, uint32_t key, int ngroups, const int *bases, const double *p) {
  if (ngroups < 1 || ngroups > 8) throw std::invalid_argument("hybrid needs 1..8 groups");
  if (dim < 2) throw std::invalid_argument("dimension must be at least 2");
  std::vector<int> sizes(ngroups);
  int used = 0;
  for (int i = 0; i + 1 < ngroups; ++i) {
    sizes[i] = static_cast<int>(std::ceil(p[i] * static_cast<double>(dim)));  // Eq. (numbers)
    used += sizes[i];
  }
  sizes[ngroups - 1] = dim - used;
  for (int i = 0; i < ngroups; ++i) {
    if (bases[i] < 0 || bases[i] > 22) throw std::invalid_argument("hybrid base id must be in 0..22");
    if (sizes[i] < min_dimension(bases[i]))
      throw std::invalid_argument("hybrid group too small for its formula (elliptic, powers and F7 need 2)");
  }
  Problem h;
  h.type = Problem::HYBRID;
  h.dim = dim;
  h.o = random_shift(seed, dim, key);
  h.orig = random_permutation(seed, dim, key);  // S
  h.rotated = true;
  h.index_by_original = false;
  Rng g(seed, dim, key, 2);
  int off = 0;
  for (int i = 0; i < ngroups; ++i) {
    const FnSpec &t = fn_spec(bases[i]);
    h.blk_off.push_back(off);
    h.blk_n.push_back(sizes[i]);
    h.Q.push_back(random_block(g, sizes[i]));
    h.segs.push_back(Segment{bases[i], off, sizes[i], t.s, t.c});
    off += sizes[i];
  }
  return h;
}

Problem make_composition(int dim, uint64_t seed, uint32_t key, int ncomp, const int *bases, const double *sigma,
                         const double *lambda, const double *bias) {
  if (ncomp < 1 || ncomp > 8) throw std::invalid_argument("composition needs 1..8 components");
  Problem q;
  q.type = Problem::COMPOSITION;
  q.dim = dim;
  for (int i = 0; i < ncomp; ++i) {
    if (bases[i] < 0 || bases[i] > 22) throw std::invalid_argument("component id must be in 0..22");
    if (!(sigma[i] > 0.0)) throw std::invalid_argument("sigma must be positive");
    const FnSpec &t = fn_spec(bases[i]);
    q.comps.push_back(make_basic(bases[i], dim, seed, key | static_cast<uint32_t>(i), t.s, t.c, t.rotated, false));
    q.sigma.push_back(sigma[i]);
    q.lambda.push_back(lambda[i]);
    q.cbias.push_back(bias[i]);
  }
  return q;
}

namespace {
// Secs. 5.1-5.6 and 6.1-6.8 parameter tables.
const int kHyN[6] = {3, 3, 4, 4, 5, 5};
const double kHyP[6][5] = {{0.3, 0.3, 0.4}, {0.3, 0.3, 0.4}, {0.2, 0.2, 0.3, 0.3},
                           {0.2, 0.2, 0.3, 0.3}, {0.1, 0.2, 0.2, 0.2, 0.3}, {0.1, 0.2, 0.2, 0.2, 0.3}};
const int kHyG[6][5] = {{15, 10, 2}, {4, 21, 10}, {9, 8, 14, 22}, {21, 3, 13, 10}, {22, 21, 14, 15, 2},
                        {17, 20, 13, 15, 19}};
const int kCoN[8] = {5, 3, 3, 5, 5, 5, 3, 3};
const double kCoSig[8][5] = {{10, 20, 30, 40, 50}, {15, 15, 15}, {20, 50, 40}, {20, 15, 10, 10, 40},
                             {15, 15, 15, 15, 15}, {10, 20, 30, 40, 50}, {10, 30, 50}, {10, 30, 50}};
const double kCoLam[8][5] = {{1e-10, 1e-6, 1e-26, 1e-6, 1e-6}, {1, 1, 1}, {0.25, 1, 1e-7},
                             {2.5e-2, 0.1, 1e-8, 0.25, 1}, {10, 10, 2.5, 2.5, 1e-6},
                             {2.5, 10, 2.5, 5e-4, 1e-6}, {1, 1, 1}, {1, 1, 1}};
const int kCoG[8][5] = {{14, 2, 4, 3, 2}, {15, 11, 21}, {16, 11, 2}, {16, 20, 2, 8, 9},
                        {21, 11, 16, 8, 2}, {13, 20, 16, 22, 2}, {23, 24, 25}, {26, 27, 28}};
}  // namespace

Problem make_tab1(int fid, int dim, uint64_t seed) {
  if (fid >= 0 && fid <= 22) return make_tab1_basic(fid, dim, seed);
  if (fid >= 23 && fid <= 28) {
    if (dim < 10) throw std::invalid_argument("hybrid functions need dim >= 10");
    int h = fid - 23;
    return make_hybrid(dim, seed, static_cast<uint32_t>(fid) << 8, kHyN[h], kHyG[h], kHyP[h]);
  }
  if (fid >= 29 && fid <= 36) {
    int c = fid - 29;
    if ((fid == 35 || fid == 36) && dim < 10) throw std::invalid_argument("hybrid components need dim >= 10");
    Problem q;
    q.type = Problem::COMPOSITION;
    q.dim = dim;
    for (int i = 0; i < kCoN[c]; ++i) {
      int g = kCoG[c][i];
      uint32_t key = (static_cast<uint32_t>(fid) << 8) | static_cast<uint32_t>(i);
      Problem comp;
      if (g >= 23) {
        int h = g - 23;
        comp = make_hybrid(dim, seed, key, kHyN[h], kHyG[h], kHyP[h]);
        if (i == 2) comp.o.assign(dim, 0.0);  // third optimum at the origin (Sec. 6)
      } else {
        const FnSpec &t = fn_spec(g);
        comp = make_basic(g, dim, seed, key, t.s, t.c, t.rotated, i == 2);
      }
      q.comps.push_back(std::move(comp));
      q.sigma.push_back(kCoSig[c][i]);
      q.lambda.push_back(kCoLam[c][i]);
      q.cbias.push_back(100.0 * i);
    }
    return q;
  }
  throw std::invalid_argument("function id must be in 0..36");
}

std::vector<double> dense_rotation(const Problem &p) {
  int D = p.dim;
  std::vector<double> R(static_cast<size_t>(D) * D, 0.0);
  if (!p.rotated) {
    for (int j = 0; j < D; ++j) R[static_cast<size_t>(j) * D + j] = 1.0;
    return R;
  }
  for (size_t k = 0; k < p.Q.size(); ++k) {
    int off = p.blk_off[k], n = p.blk_n[k];
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b)
        R[static_cast<size_t>(p.orig[off + a]) * D + p.orig[off + b]] = p.Q[k][static_cast<size_t>(a) * n + b];
  }
  return R;
}

double formula_coef(int base, int i, int n) {
  switch (base) {
    case 0: return 1.0;
    case 1: return static_cast<double>(i + 1);
    case 2: return std::pow(1.0e6, static_cast<double>(i) / static_cast<double>(n - 1));
    case 3: return i == 0 ? 1.0e6 : 1.0;
    case 4: return i == 0 ? 1.0 : 1.0e6;
    case 5: return 2.0 + 4.0 * static_cast<double>(i) / static_cast<double>(n - 1);
    case 6: return i == 0 ? 1.0 : 0.0;
    case 9: return 1.0 / std::sqrt(static_cast<double>(i + 1));
    case 17: return static_cast<double>(i + 1);
    default: return 0.0;
  }
}

}  // namespace curob
