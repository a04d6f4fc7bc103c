// formulas.h -- device side of the cuROB formulas (Secs. 3-4): per-element terms and the
// per-row finalisation, templated on float / double.
#pragma once

#include <hip/hip_runtime.h>

#include "problem.h"
#include "schwefel_series.h"

namespace curob {

// Up to three sums and one product per row.  Terms are first added plainly in groups of four
// (one accumulator fragment); the group sums then enter a running FP32 sum that is
// Kahan-compensated for the families whose terms have mixed signs and can cancel (Weierstrass,
// Schwefel, Ackley's cosine sum, Lunacek, HappyCat, HGBat; KindTraits::kahan).  What padded
// positions added is removed before the compensation is folded in (Acc::get_minus).  Sums of non-negative terms (sphere family
// including the 1e6-weighted elliptic, Rastrigin, Rosenbrock, Griewank, step, ...) are added
// plainly: with no cancellation the relative error of an n-term FP32 sum stays below
// n x 2^-24 (6e-6 at n = 100, 6e-5 at n = 1000, against the 1e-4 bar), and the lanes' partial
// sums are merged with TwoSum, which keeps that bound.  FP64 sums are plain.
template <typename T>
struct Acc {
  T s[3];
  T c[3];
  T p;
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int k = 0; k < 3; ++k) s[k] = c[k] = T(0);
    p = T(1);
  }
  __device__ __forceinline__ void add(int k, T v) {
    if constexpr (sizeof(T) == 4) {
      T y = v - c[k];
      T t = s[k] + y;
      c[k] = (t - s[k]) - y;
      s[k] = t;
    } else {
      s[k] += v;
    }
  }
  __device__ __forceinline__ T get(int k) const { return s[k] - c[k]; }
  // The sum minus a constant d (what padded positions added), taken before the compensation
  // is folded in: when the sum and d nearly cancel, s - d_hi is exact (Sterbenz) and the
  // compensation and the rounding remainder of d survive, instead of vanishing in the rounding
  // of s - c to the sum's own ulp.
  __device__ __forceinline__ T get_minus(int k, double d) const {
    const T dh = T(d);
    const T dl = T(d - static_cast<double>(dh));
    return ((s[k] - dh) - c[k]) - dl;
  }
};


// FP64 cos(2 pi t) for t in [-1/2, 1/2], branch free: cos(2 pi t) = -cos(2 pi (1/2 - |t|))
// folds t onto [0, 1/4], where x = 2 pi t <= pi/2 and the Taylor series of cos in x^2 up to the
// x^22 term leaves a truncation error below 2e-17 (the next term is x^24 / 24!).  Horner in x^2
// with fused multiply-adds; measured against a long-double reference: <= 7e-16 absolute.
__device__ __forceinline__ double cos2pi_reduced(double t) {
  const double a = __builtin_fabs(t);
  const bool far = a > 0.25;
  const double u = far ? 0.5 - a : a;  // exact for a in (1/4, 1/2]
  const double x = 6.283185307179586477 * u;
  const double y = x * x;
  double p = -1.0 / 51090942171709440000.0;  // -1/22!
  p = __builtin_fma(p, y, 1.0 / 2432902008176640000.0);  // 1/20!
  p = __builtin_fma(p, y, -1.0 / 6402373705728000.0);    // -1/18!
  p = __builtin_fma(p, y, 1.0 / 20922789888000.0);       // 1/16!
  p = __builtin_fma(p, y, -1.0 / 87178291200.0);         // -1/14!
  p = __builtin_fma(p, y, 1.0 / 479001600.0);            // 1/12!
  p = __builtin_fma(p, y, -1.0 / 3628800.0);             // -1/10!
  p = __builtin_fma(p, y, 1.0 / 40320.0);                // 1/8!
  p = __builtin_fma(p, y, -1.0 / 720.0);                 // -1/6!
  p = __builtin_fma(p, y, 1.0 / 24.0);                   // 1/4!
  p = __builtin_fma(p, y, -0.5);                         // -1/2!
  p = __builtin_fma(p, y, 1.0);
  return far ? -p : p;
}

// cos(2 pi z) with the argument reduced exactly: z - rint(z) is exact in binary floating point.
__device__ __forceinline__ float cos_2pi(float z) { return __builtin_amdgcn_cosf(z - rintf(z)); }
__device__ __forceinline__ double cos_2pi(double z) { return cos2pi_reduced(z - rint(z)); }

// sin(x) for x in radians: x/(2 pi) in revolutions (one rounding, whose relative error bounds
// the phase error), reduced exactly.  FP32: the hardware sine; FP64: sin x = cos(x - pi/2).
__device__ __forceinline__ float sin_rad(float x) {
  float t = x * 0.15915494309189535f;
  return __builtin_amdgcn_sinf(t - rintf(t));
}
__device__ __forceinline__ double sin_rad(double x) {
  const double t = __builtin_fma(x, 0.15915494309189533577, -0.25);
  return cos2pi_reduced(t - rint(t));
}

// cos of an argument given in revolutions: the Griewank coefficient table holds 1/(2 pi sqrt(i)).
__device__ __forceinline__ float cos_scaled(float t) { return __builtin_amdgcn_cosf(t - rintf(t)); }
__device__ __forceinline__ double cos_scaled(double t) { return cos2pi_reduced(t - rint(t)); }

template <typename T>
__device__ __forceinline__ T t_sqrt(T v) {
  if constexpr (sizeof(T) == 4) return __builtin_sqrtf(v); else return __builtin_sqrt(v);
}
template <typename T>
__device__ __forceinline__ T t_pow(T a, T b) {
  if constexpr (sizeof(T) == 4) return powf(a, b); else return pow(a, b);
}
template <typename T>
__device__ __forceinline__ T t_exp(T v) {
  if constexpr (sizeof(T) == 4) return expf(v); else return exp(v);
}
template <typename T>
__device__ __forceinline__ T t_floor(T v) {
  if constexpr (sizeof(T) == 4) return __builtin_floorf(v); else return __builtin_floor(v);
}
template <typename T>
__device__ __forceinline__ T t_rint(T v) {
  if constexpr (sizeof(T) == 4) return __builtin_rintf(v); else return __builtin_rint(v);
}
template <typename T>
__device__ __forceinline__ T t_abs(T v) {
  if constexpr (sizeof(T) == 4) return __builtin_fabsf(v); else return __builtin_fabs(v);
}

// One Schwefel term 418.9829 - g1(z + w*) of Eq. (basic_schwefel), branch free, w* =
// 420.9687....  With w = z + w* and a = |w|: for a <= 500 g1 is w sin(sqrt a); beyond, both outer
// branches fold a back to u = 500 - mod(a, 500) and subtract (a - 500)^2 / (10000 n):
// g1 = sign(w) u sin(sqrt u) - penalty.  Summing 418.9829 - g1 per term (the function is the sum
// of these) keeps the terms small near the optimum, where 418.9829 n and the sum of g1 would cancel
// to the ulp of 418.9829 n.  In FP32 the constant is fl32(418.9829), the finalisation adds
// n (418.9829 - fl32(418.9829)), and within |z| < 4 of the optimum the term comes from the fitted
// series of schwefel_series.h: every term of a row at the optimum shares one argument, so the
// direct form's roundings of sqrt, phase and sine (~4e-5 per term) would add up over the row.
template <typename T>
__device__ __forceinline__ T schwefel_g1(T z, T inv10000n) {
  if constexpr (sizeof(T) == 4) {
    const float w = z + static_cast<float>(kSchwefelW);
    const float a = __builtin_fabsf(w);
    const bool far = a > 500.0f;
    // mod(a, 500) as 500 fract(a / 500): a few ulps of a from the exact remainder, which
    // only moves the jumps at a = 1000, 1500, ... by as much
    const float m = 500.0f * __builtin_amdgcn_fractf(a * 0.002f);
    const float u = far ? 500.0f - m : a;
    const float d = __builtin_fmaxf(a - 500.0f, 0.0f);
    // sqrt(u) <= sqrt(500) < 23: the sine's argument in revolutions stays below 4, inside
    // the hardware sine's domain, so no range reduction is needed.  The hardware square root
    // (1 ulp) moves the phase by at most 23 x 2^-23 rad, the order of the revolution rounding.
    const float sn = __builtin_amdgcn_sinf(__builtin_amdgcn_sqrtf(u) * 0.15915494309189535f);
    // C - g1 with the product rounded once
    const float direct = __builtin_fmaf(-__builtin_copysignf(u, w), sn, static_cast<float>(kSchwefelC)) + d * d * inv10000n;
    const float t = z * kSchwefelInvRho;
    float q = kSchwefelQ[3];
#pragma unroll
    for (int j = 2; j >= 0; --j) q = __builtin_fmaf(q, t, kSchwefelQ[j]);
    const float series = __builtin_fmaf(z * z, q, kSchwefelT0);
    return __builtin_fabsf(z) < kSchwefelRho ? series : direct;
  } else {
    const T w = z + T(kSchwefelW);
    const T a = t_abs(w);
    const bool far = a > T(500);
    T m = a - T(500) * t_floor(a * T(0.002));  // mod(a, 500); the floor may be off by one
    m = m < T(0) ? m + T(500) : m;
    m = m >= T(500) ? m - T(500) : m;
    const T u = far ? T(500) - m : a;
    const T d = a - T(500);
    const T pen = far ? d * d * inv10000n : T(0);
    const T g = u * sin_rad(t_sqrt(u));
    return T(kSchwefelC) - (w < T(0) ? -g : g) + pen;
  }
}

template <int KIND>
struct KindTraits {
  static constexpr bool pairwise = KIND == K_F7 || KIND == K_GRIEROSEN || KIND == K_ROSENBROCK || KIND == K_F6;
  static constexpr bool needs_coef = KIND == K_WSPHERE || KIND == K_POWERS || KIND == K_SHARPV ||
                                     KIND == K_GRIEWANK || KIND == K_KATSUURA;
  static constexpr bool has_product = KIND == K_GRIEWANK || KIND == K_KATSUURA;
  // Sums whose terms can cancel (mixed signs) are Kahan-compensated in FP32; sums of
  // non-negative terms are added plainly: their relative error stays below (terms) x 2^-24.
  static constexpr bool kahan = KIND == K_WEIERSTRASS || KIND == K_SCHWEFEL || KIND == K_ACKLEY ||
                                KIND == K_LUNACEK || KIND == K_HAPPYCAT || KIND == K_HGBAT;
  // sums the family keeps per row
  static constexpr int nsum = (KIND == K_LUNACEK) ? 3
                              : (KIND == K_SHARPV || KIND == K_ACKLEY || KIND == K_HAPPYCAT || KIND == K_HGBAT) ? 2
                              : (KIND == K_KATSUURA) ? 0
                                                     : 1;
};

// Adds a group sum to a row sum: compensated where the family's sums can cancel.
template <int KIND, typename T>
__device__ __forceinline__ void acc_add(Acc<T> &a, int k, T v) {
  if constexpr (KindTraits<KIND>::kahan) a.add(k, v);
  else a.s[k] += v;
}

// Adds the term(s) of one element z (with its formula successor zn for the pairwise
// families) to the group sums v[] and the product p.  `prm` carries the row-independent
// parameter (1/(10000 n) for Schwefel, the Katsuura exponent).
template <int KIND, typename T>
__device__ __forceinline__ void phi(T (&v)[3], T &p, T z, T zn, T coef, T prm) {
  if constexpr (KIND == K_WSPHERE) {
    v[0] += coef * z * z;
  } else if constexpr (KIND == K_POWERS) {
    v[0] += t_pow(t_abs(z), coef);
  } else if constexpr (KIND == K_SHARPV) {
    const T q = z * z;
    v[0] += coef * q;
    v[1] += (T(1) - coef) * q;
  } else if constexpr (KIND == K_STEP) {
    const T f = t_floor(z + T(0.5));
    v[0] += f * f;
  } else if constexpr (KIND == K_WEIERSTRASS) {
    const T u = z + T(0.5);
    T acc = T(0), ak = T(1), bk = T(1);
#pragma unroll
    for (int k = 0; k <= 20; ++k) {
      acc += ak * cos_2pi(bk * u);
      ak *= T(0.5);
      bk *= T(3);
    }
    v[0] += acc;
  } else if constexpr (KIND == K_GRIEWANK) {
    v[0] += z * z;
    p *= cos_scaled(z * coef);
  } else if constexpr (KIND == K_RASTRIGIN) {
    v[0] += z * z + T(10) * (T(1) - cos_2pi(z));
  } else if constexpr (KIND == K_F7) {
    const T w = t_sqrt(z * z + zn * zn);
    const T sn = sin_rad(T(50) * t_pow(w, T(0.2)));
    v[0] += (T(1) + sn * sn) * t_sqrt(w);
  } else if constexpr (KIND == K_GRIEROSEN) {
    const T d = z * z - zn;
    const T e = z - T(1);
    const T g2 = T(100) * d * d + e * e;
    T cg;
    // FP32: g2 / (2 pi) in revolutions, reduced exactly, then the hardware cosine.  The phase
    // error is the rounding of g2 / (2 pi), 2^-24 g2, while f grows as g2^2 / 4000: the cosine
    // error stays far below the FP32 bar for every g2
    if constexpr (sizeof(T) == 4) cg = cos_2pi(g2 * 0.15915494309189535f); else cg = cos(g2);
    v[0] += g2 * g2 * T(1.0 / 4000.0) - cg + T(1);
  } else if constexpr (KIND == K_ROSENBROCK) {
    const T d = z * z - zn;
    const T e = z - T(1);
    v[0] += T(100) * d * d + e * e;
  } else if constexpr (KIND == K_SCHWEFEL) {
    v[0] += schwefel_g1(z, prm);
  } else if constexpr (KIND == K_KATSUURA) {
    T t = T(0), pj = T(1);
#pragma unroll 4
    for (int j = 1; j <= 32; ++j) {
      pj *= T(2);
      const T q = pj * z;
      t += t_abs(q - t_rint(q)) / pj;
    }
    p *= t_pow(T(1) + coef * t, prm);
  } else if constexpr (KIND == K_LUNACEK) {
    const T u = z - T(2.5), w = z + T(2.5);
    v[0] += u * u;
    v[1] += w * w;
    v[2] += cos_2pi(u);
  } else if constexpr (KIND == K_ACKLEY) {
    v[0] += z * z;
    v[1] += cos_2pi(z);
  } else if constexpr (KIND == K_HAPPYCAT) {
    // on w = z + 1: z^2 - 1 = w (w - 2) and z = w - 1.  Near the optimum w -> 0 and these
    // terms keep their relative precision, where sum z^2 - n cancels to ulps of n
    v[0] += z * (z - T(2));
    v[1] += z;
  } else if constexpr (KIND == K_HGBAT) {
    // on w = z + 1: (sum z^2)^2 - (sum z)^2 = sum(z^2 + z) sum(z^2 - z) with z^2 + z = w (w - 1)
    // and z^2 - z = (w - 1)(w - 2).  Near the optimum the first factor is small and stays
    // accurate (the two squares, each ~n^2, would cancel)
    v[0] += z * (z - T(1));
    v[1] += (z - T(1)) * (z - T(2));
  } else if constexpr (KIND == K_F6) {
    const T r2 = z * z + zn * zn;
    const T sn = sin_rad(t_sqrt(r2));
    const T den = T(1) + T(0.001) * r2;
    v[0] += (sn * sn - T(0.5)) / (den * den) + T(0.5);
  }
}

// Row value (without f_opt) from the combined sums s[k] (padding already removed) and
// product p; n = dimension the formula sees.
template <int KIND, typename T>
__device__ __forceinline__ T finalize(const T (&s)[3], T p, int n) {
  const T nn = T(n);
  if constexpr (KIND == K_WSPHERE || KIND == K_STEP || KIND == K_RASTRIGIN || KIND == K_GRIEROSEN ||
                KIND == K_ROSENBROCK || KIND == K_F6) {
    return s[0];
  } else if constexpr (KIND == K_POWERS) {
    return t_sqrt(s[0]);
  } else if constexpr (KIND == K_SHARPV) {
    return s[0] + T(100) * t_sqrt(s[1]);
  } else if constexpr (KIND == K_WEIERSTRASS) {
    // each cos(pi 3^k) is -1, so the constant term is -n (2 - 2^-20)
    return s[0] + nn * T(2.0 - 9.5367431640625e-07);
  } else if constexpr (KIND == K_GRIEWANK) {
    return s[0] * T(1.0 / 4000.0) - p + T(1);
  } else if constexpr (KIND == K_F7) {
    const T t = s[0] / (nn - T(1));
    return t * t;
  } else if constexpr (KIND == K_SCHWEFEL) {
    // s[0] = sum (C - g1) with C = 418.9829 rounded to T
    return s[0] + nn * T(kSchwefelC - static_cast<double>(T(kSchwefelC)));
  } else if constexpr (KIND == K_KATSUURA) {
    const T c = T(10) / (nn * nn);
    return c * p - c;
  } else if constexpr (KIND == K_LUNACEK) {
    const T first = s[0], second = nn + T(0.9) * s[1];
    return (first < second ? first : second) + T(10) * (nn - s[2]);
  } else if constexpr (KIND == K_ACKLEY) {
    return T(-20) * t_exp(T(-0.2) * t_sqrt(s[0] / nn)) - t_exp(s[1] / nn) + T(20) + T(2.71828182845904523536);
  } else if constexpr (KIND == K_HAPPYCAT) {
    // s[0] = sum(z^2 - 1) = sum z^2 - n, s[1] = sum w = sum z + n:
    // (0.5 sum z^2 + sum z) / n + 0.5 = (0.5 s[0] + s[1]) / n
    return t_pow(t_abs(s[0]), T(0.25)) + (T(0.5) * s[0] + s[1]) / nn;
  } else if constexpr (KIND == K_HGBAT) {
    // s[0] = sum(z^2 + z), s[1] = sum(z^2 - z): sum z^2 = (s0 + s1)/2, sum z = (s0 - s1)/2
    return t_sqrt(t_abs(s[0] * s[1])) + (T(0.75) * s[0] - T(0.25) * s[1]) / nn + T(0.5);
  } else {
    return T(0);
  }
}

// Pairwise families whose last term pairs z_n with z_1 (device-side copy of the host rule).
__host__ __device__ constexpr bool kind_pair_wraps_c(int kind) { return kind == K_GRIEROSEN || kind == K_F6; }

// Parameter passed to phi for each family.
template <int KIND, typename T>
__device__ __forceinline__ T kind_param(int n, double kparam) {
  if constexpr (KIND == K_SCHWEFEL) return T(1.0 / (10000.0 * (double)n));
  else if constexpr (KIND == K_KATSUURA) return T(kparam);
  else return T(0);
}

// Combine another lane's compensated state (s, c) into a: TwoSum of the leading parts, the
// rounding error joins the compensation.
template <typename T>
__device__ __forceinline__ void acc_merge(Acc<T> &a, int k, T s, T c) {
  if constexpr (sizeof(T) == 4) {
    const T t = a.s[k] + s;
    const T bp = t - a.s[k];
    const T err = (a.s[k] - (t - bp)) + (s - bp);
    a.s[k] = t;
    a.c[k] = a.c[k] + c - err;
  } else {
    a.s[k] += s;
  }
}

}  // namespace curob
