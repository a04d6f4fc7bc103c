"""The FP32 kernels' series for one modified-Schwefel term near the optimum of g1 (Sec. 4.9):
the committed header is what its generator writes, and the series, evaluated in FP32 the way
the kernels do, stays within FP32 rounding of the term's FP64 definition
C - (w* + z) sin(sqrt(w* + z)) with C = fl32(418.9829), the constant of the kernels' other terms."""
import importlib.util
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GEN = os.path.join(ROOT, "paper_1407_7737_amd", "csrc", "schwefel_series.py")


def load_gen():
    spec = importlib.util.spec_from_file_location("schwefel_series", GEN)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_header_is_generated():
    gen = load_gen()
    with open(gen.HEADER) as fh:
        assert fh.read() == gen.header_text()


def test_series_in_fp32_matches_the_term():
    gen = load_gen()
    t0, q = gen.fit()
    t0f, qf = np.float32(t0), q.astype(np.float32)
    rho = np.float32(gen.RHO)
    inv = np.float32(1.0 / gen.RHO)
    w_star = 420.9687462275036
    # z = w - w* in FP32 as the rotation delivers it, over the series' range and densely near 0
    z = np.concatenate([np.linspace(-float(rho), float(rho), 200001), np.linspace(-1e-3, 1e-3, 2001)]).astype(np.float32)
    z = z[np.abs(z) < rho]
    t = (z * inv).astype(np.float32)
    acc = np.full_like(t, qf[-1])
    for c in qf[-2::-1]:
        acc = (acc * t + c).astype(np.float32)  # FP32 Horner (the kernels fuse each step)
    val = ((z * z).astype(np.float32) * acc + t0f).astype(np.float32).astype(np.float64)
    exact = gen.C_F32 - (w_star + z.astype(np.float64)) * np.sin(np.sqrt(w_star + z.astype(np.float64)))
    err = np.abs(val - exact)
    assert err.max() <= 1e-6
    near = np.abs(z) < 1e-3
    assert near.any() and err[near].max() <= 1e-10
    # relative to the term wherever it is not tiny
    big = exact > 1e-3
    assert (err[big] / exact[big]).max() <= 1e-5


def test_value_at_the_optimum():
    """T(0) + 418.9829 - fl32(418.9829) = 418.9829 - w* sin(sqrt(w*)): the per-variable offset of
    f(x_opt) above f_opt."""
    gen = load_gen()
    t0, _ = gen.fit()
    assert abs(t0 + (418.9829 - gen.C_F32) - 1.2727566173e-5) <= 1e-15
