// schwefel_series.h -- written by schwefel_series.py (do not edit): one modified-Schwefel
// term fl32(418.9829) - g1(w* + z) near the optimum w* = 420.9687462275036 of g1 (Sec. 4.9) as
// T0 + z^2 Q(z / 4) for |z| < 4; Q fitted in FP64 (degree 3, least squares on
// 400 Chebyshev nodes).
#pragma once

namespace curob {

constexpr float kSchwefelRho = 4.0f;
constexpr float kSchwefelInvRho = 0.25f;
constexpr float kSchwefelT0 = 2.2883816200192086e-05f;
constexpr float kSchwefelQ[4] = {0.12618352472782135f, 0.00019414736016187817f, -0.0001015115121845156f, 2.7045322781305003e-07f};

}  // namespace curob
