"""Writes schwefel_series.h: the FP32 kernels' polynomial for one modified-Schwefel term near
the optimum of g1 (Sec. 4.9).

The term is T(z) = C - g1(w* + z) with w* = 420.9687462275036 and C = 418.9829 (both printed in
the paper) rounded to FP32 as the kernels' other terms use it (their row finalisation adds
n (418.9829 - C)), and g1(w) = w sin(sqrt(w)) for 0 < w <= 500.  g1 is stationary at w*, so near it T(z) is
T(0) + O(z^2).  Evaluated directly in FP32, every intermediate (sqrt(w), the phase, the sine)
is rounded at the scale of w ~ 421, and since all terms of a row at the optimum share the same
argument those roundings add up instead of averaging out.  For |z| < RHO the kernels instead
evaluate T(z) = T(0) + z^2 Q(z / RHO), with Q a polynomial fitted here in FP64 by least
squares on Chebyshev nodes.  tests/test_schwefel_series.py checks the header against this
script and the polynomial against T in FP32.

    python paper_1407_7737_amd/csrc/schwefel_series.py    # rewrites schwefel_series.h
"""
import os

import numpy as np

W_OPT = 420.9687462275036  # Sec. 4.9
C_SCHWEFEL = 418.9829      # Sec. 4.9
C_F32 = float(np.float32(C_SCHWEFEL))  # the constant as the FP32 kernels hold it
RHO = 4.0                  # |z| below which the polynomial is used
DEGREE = 3                 # degree of Q
NODES = 400

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = os.path.join(HERE, "schwefel_series.h")


def term(z):
    """T(z) = fl32(418.9829) - g1(w* + z) in FP64 (0 < w* + z <= 500)."""
    w = W_OPT + np.asarray(z, dtype=np.float64)
    return C_F32 - w * np.sin(np.sqrt(w))


def fit():
    """(T(0), coefficients of Q in increasing order) in FP64."""
    u = np.cos(np.pi * (np.arange(NODES) + 0.5) / NODES)
    z = RHO * u
    t0 = float(term(0.0))
    q = (term(z) - t0) / (z * z)
    return t0, np.polynomial.polynomial.polyfit(u, q, DEGREE)


def f32(v: float) -> str:
    """A decimal literal that rounds to the nearest FP32 value of v."""
    return repr(float(np.float32(v))) + "f"


def header_text() -> str:
    t0, q = fit()
    lines = [
        "// schwefel_series.h -- written by schwefel_series.py (do not edit): one modified-Schwefel",
        "// term fl32(418.9829) - g1(w* + z) near the optimum w* = 420.9687462275036 of g1 (Sec. 4.9) as",
        f"// T0 + z^2 Q(z / {RHO:g}) for |z| < {RHO:g}; Q fitted in FP64 (degree {DEGREE}, least squares on",
        f"// {NODES} Chebyshev nodes).",
        "#pragma once",
        "",
        "namespace curob {",
        "",
        f"constexpr float kSchwefelRho = {f32(RHO)};",
        f"constexpr float kSchwefelInvRho = {f32(1.0 / RHO)};",
        f"constexpr float kSchwefelT0 = {f32(t0)};",
        f"constexpr float kSchwefelQ[{DEGREE + 1}] = {{" + ", ".join(f32(c) for c in q) + "};",
        "",
        "}  // namespace curob",
        "",
    ]
    return "\n".join(lines)


if __name__ == "__main__":
    with open(HEADER, "w") as fh:
        fh.write(header_text())
    print(HEADER)
