// formulas.h -- device side of the cuROB formulas (Secs. 3-4): per-element terms and the
// per-row finalisation, templated on float / double.
#pragma once

#include <hip/hip_runtime.h>

#include "problem.h"

namespace curob {

// Compensated accumulators for up to three sums and one product per row.  FP32 sums use
// Kahan's compensation (the elliptic weights span six decades and the Rastrigin terms reach
// 1e4 at |z| ~ 100, so plain FP32 sums would lose digits); FP64 sums are plain.
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
};

// cos(2 pi z) with the argument reduced exactly: z - rint(z) is exact in binary floating point.
__device__ __forceinline__ float cos_2pi(float z) { return __builtin_amdgcn_cosf(z - rintf(z)); }
__device__ __forceinline__ double cos_2pi(double z) { return cospi(2.0 * (z - rint(z))); }

// sin(x) for x in radians.  FP32: x/(2 pi) in revolutions, reduced exactly, then the hardware
// sine; the relative error of the one rounding of x/(2 pi) bounds the phase error.
__device__ __forceinline__ float sin_rad(float x) {
  float t = x * 0.15915494309189535f;
  return __builtin_amdgcn_sinf(t - rintf(t));
}
__device__ __forceinline__ double sin_rad(double x) { return sin(x); }

// cos(x) with x given in revolutions (FP32) or radians (FP64): the Griewank coefficient
// table holds 1/(2 pi sqrt(i)) for FP32 and 1/sqrt(i) for FP64.
__device__ __forceinline__ float cos_scaled(float t) { return __builtin_amdgcn_cosf(t - rintf(t)); }
__device__ __forceinline__ double cos_scaled(double x) { return cos(x); }

template <typename T>
__device__ __forceinline__ T t_sqrt(T v) {
  if constexpr (sizeof(T) == 4) return sqrtf(v); else return sqrt(v);
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
  if constexpr (sizeof(T) == 4) return floorf(v); else return floor(v);
}
template <typename T>
__device__ __forceinline__ T t_rint(T v) {
  if constexpr (sizeof(T) == 4) return rintf(v); else return rint(v);
}
template <typename T>
__device__ __forceinline__ T t_fmod(T a, T b) {
  if constexpr (sizeof(T) == 4) return fmodf(a, b); else return fmod(a, b);
}

// Modified Schwefel g1 of Eq. (basic_schwefel), n the dimension the formula sees.
template <typename T>
__device__ __forceinline__ T schwefel_g1(T w, T inv10000n) {
  T aw = w < T(0) ? -w : w;
  if (aw <= T(500)) return w * sin_rad(t_sqrt(aw));
  if (w > T(500)) {
    T m = t_fmod(w, T(500));
    T d = w - T(500);
    return (T(500) - m) * sin_rad(t_sqrt(T(500) - m)) - d * d * inv10000n;
  }
  T m = t_fmod(-w, T(500));
  T d = w + T(500);
  return (m - T(500)) * sin_rad(t_sqrt(T(500) - m)) - d * d * inv10000n;
}

template <int KIND>
struct KindTraits {
  static constexpr bool pairwise = KIND == K_F7 || KIND == K_GRIEROSEN || KIND == K_ROSENBROCK || KIND == K_F6;
  static constexpr bool needs_coef = KIND == K_WSPHERE || KIND == K_POWERS || KIND == K_SHARPV ||
                                     KIND == K_GRIEWANK || KIND == K_KATSUURA;
};

// Term of one element z (with its formula successor zn for the pairwise families).
// `prm` carries the row-independent parameters (1/(10000 n) for Schwefel, the Katsuura exponent).
template <int KIND, typename T>
__device__ __forceinline__ void phi(Acc<T> &a, T z, T zn, T coef, T prm) {
  if constexpr (KIND == K_WSPHERE) {
    a.add(0, coef * z * z);
  } else if constexpr (KIND == K_POWERS) {
    T az = z < T(0) ? -z : z;
    a.add(0, t_pow(az, coef));
  } else if constexpr (KIND == K_SHARPV) {
    if (coef != T(0)) a.add(0, z * z); else a.add(1, z * z);
  } else if constexpr (KIND == K_STEP) {
    T f = t_floor(z + T(0.5));
    a.add(0, f * f);
  } else if constexpr (KIND == K_WEIERSTRASS) {
    T u = z + T(0.5);
    T acc = T(0), ak = T(1), bk = T(1);
#pragma unroll
    for (int k = 0; k <= 20; ++k) {
      acc += ak * cos_2pi(bk * u);
      ak *= T(0.5);
      bk *= T(3);
    }
    a.add(0, acc);
  } else if constexpr (KIND == K_GRIEWANK) {
    a.add(0, z * z);
    a.p *= cos_scaled(z * coef);
  } else if constexpr (KIND == K_RASTRIGIN) {
    a.add(0, z * z + T(10) * (T(1) - cos_2pi(z)));
  } else if constexpr (KIND == K_F7) {
    T w = t_sqrt(z * z + zn * zn);
    T sn = sin_rad(T(50) * t_pow(w, T(0.2)));
    a.add(0, (T(1) + sn * sn) * t_sqrt(w));
  } else if constexpr (KIND == K_GRIEROSEN) {
    T d = z * z - zn;
    T e = z - T(1);
    T g2 = T(100) * d * d + e * e;
    T cg;
    if constexpr (sizeof(T) == 4) cg = cosf(g2); else cg = cos(g2);
    a.add(0, g2 * g2 / T(4000) - cg + T(1));
  } else if constexpr (KIND == K_ROSENBROCK) {
    T d = z * z - zn;
    T e = z - T(1);
    a.add(0, T(100) * d * d + e * e);
  } else if constexpr (KIND == K_SCHWEFEL) {
    a.add(0, schwefel_g1(z + T(420.9687462275036), prm));
  } else if constexpr (KIND == K_KATSUURA) {
    T t = T(0), pj = T(1);
#pragma unroll 4
    for (int j = 1; j <= 32; ++j) {
      pj *= T(2);
      T v = pj * z;
      T d = v - t_rint(v);
      t += (d < T(0) ? -d : d) / pj;
    }
    a.p *= t_pow(T(1) + coef * t, prm);
  } else if constexpr (KIND == K_LUNACEK) {
    T u = z - T(2.5), v = z + T(2.5);
    a.add(0, u * u);
    a.add(1, v * v);
    a.add(2, cos_2pi(u));
  } else if constexpr (KIND == K_ACKLEY) {
    a.add(0, z * z);
    a.add(1, cos_2pi(z));
  } else if constexpr (KIND == K_HAPPYCAT || KIND == K_HGBAT) {
    a.add(0, z * z);
    a.add(1, z);
  } else if constexpr (KIND == K_F6) {
    T r2 = z * z + zn * zn;
    T sn = sin_rad(t_sqrt(r2));
    T den = T(1) + T(0.001) * r2;
    a.add(0, (sn * sn - T(0.5)) / (den * den) + T(0.5));
  }
}

// Row value (without f_opt) from the combined accumulators; n = dimension the formula sees.
template <int KIND, typename T>
__device__ __forceinline__ T finalize(const Acc<T> &a, int n) {
  const T nn = T(n);
  if constexpr (KIND == K_WSPHERE || KIND == K_STEP || KIND == K_RASTRIGIN || KIND == K_GRIEROSEN ||
                KIND == K_ROSENBROCK || KIND == K_F6) {
    return a.get(0);
  } else if constexpr (KIND == K_POWERS) {
    return t_sqrt(a.get(0));
  } else if constexpr (KIND == K_SHARPV) {
    return a.get(0) + T(100) * t_sqrt(a.get(1));
  } else if constexpr (KIND == K_WEIERSTRASS) {
    // each cos(pi 3^k) is -1, so the constant term is -n (2 - 2^-20)
    return a.get(0) + nn * T(2.0 - 9.5367431640625e-07);
  } else if constexpr (KIND == K_GRIEWANK) {
    return a.get(0) / T(4000) - a.p + T(1);
  } else if constexpr (KIND == K_F7) {
    T t = a.get(0) / (nn - T(1));
    return t * t;
  } else if constexpr (KIND == K_SCHWEFEL) {
    return T(418.9829) * nn - a.get(0);
  } else if constexpr (KIND == K_KATSUURA) {
    T c = T(10) / (nn * nn);
    return c * a.p - c;
  } else if constexpr (KIND == K_LUNACEK) {
    T first = a.get(0), second = nn + T(0.9) * a.get(1);
    return (first < second ? first : second) + T(10) * (nn - a.get(2));
  } else if constexpr (KIND == K_ACKLEY) {
    return T(-20) * t_exp(T(-0.2) * t_sqrt(a.get(0) / nn)) - t_exp(a.get(1) / nn) + T(20) +
           T(2.71828182845904523536);
  } else if constexpr (KIND == K_HAPPYCAT) {
    T s2 = a.get(0), s1 = a.get(1);
    T d = s2 - nn;
    return t_pow(d < T(0) ? -d : d, T(0.25)) + (T(0.5) * s2 + s1) / nn + T(0.5);
  } else if constexpr (KIND == K_HGBAT) {
    // (sum z^2)^2 - (sum z)^2 factored as (a - |b|)(a + |b|): near the optimum both squares
    // are ~n^2 and their FP32 difference would cancel to a few ulps of n^2
    T s2 = a.get(0), s1 = a.get(1);
    T b = s1 < T(0) ? -s1 : s1;
    T d = (s2 - b) * (s2 + b);
    return t_sqrt(d < T(0) ? -d : d) + (T(0.5) * s2 + s1) / nn + T(0.5);
  } else {
    return T(0);
  }
}

// Parameter passed to phi for each family.
template <int KIND, typename T>
__device__ __forceinline__ T kind_param(int n, double kparam) {
  if constexpr (KIND == K_SCHWEFEL) return T(1.0 / (10000.0 * (double)n));
  else if constexpr (KIND == K_KATSUURA) return T(kparam);
  else return T(0);
}

// Combine two Kahan states exactly up to the final rounding (TwoSum of the leading parts).
template <typename T>
__device__ __forceinline__ void acc_merge(Acc<T> &a, const T (&s)[3], const T (&c)[3], T p) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if constexpr (sizeof(T) == 4) {
      T t = a.s[k] + s[k];
      T bp = t - a.s[k];
      T err = (a.s[k] - (t - bp)) + (s[k] - bp);
      a.s[k] = t;
      a.c[k] = a.c[k] + c[k] - err;
    } else {
      a.s[k] += s[k];
    }
  }
  a.p *= p;
}

}  // namespace curob
