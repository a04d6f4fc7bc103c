// schwefel_series.h -- written by schwefel_series.py (do not edit): one modified-Schwefel
// term fl32(418.9829) - g1(w* + z) near the optimum w* = 420.9687462275036 of g1 (Sec. 4.9) as
// T0 + z^2 Q(z / 6) for |z| < 6; Q fitted in FP64 (degree 5, least squares on
// 400 Chebyshev nodes).
#pragma once

namespace curob {

constexpr float kSchwefelRho = 6.0f;
constexpr float kSchwefelInvRho = 0.1666666716337204f;
constexpr float kSchwefelT0 = 2.2883816200192086e-05f;
constexpr float kSchwefelQ[6] = {0.12618352472782135f, 0.00029122093110345304f, -0.00022847234504297376f, 9.55416908254847e-07f, 1.6078497822036297e-07f, -1.7983208522309724e-07f};

}  // namespace curob
