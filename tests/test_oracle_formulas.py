"""Pins for the oracle's formulas (Secs. 3-4, Tab. 1).

Closed-form values at exact points, the optimum f(x_opt) = f_opt of Sec. 1.2, lower bounds on
random points, transform orientation checks and a D = 2 brute-force grid search.
"""
import math

import numpy as np
import pytest

F_OPT = 100.0
# w sin(sqrt(w)) at w = 420.9687462275036 is 418.98288727..., a little below the printed
# constant 418.9829, so the modified Schwefel value at x_opt exceeds f_opt by this much per dimension.
SCHWEFEL_OFFSET_PER_DIM = 418.9829 - 420.9687462275036 * math.sin(math.sqrt(420.9687462275036))
ALL_BASIC = list(range(23))


def test_schwefel_offset_value():
    assert abs(SCHWEFEL_OFFSET_PER_DIM - 1.2727566173e-5) < 1e-14


@pytest.mark.parametrize("dim", [2, 10, 30, 100])
@pytest.mark.parametrize("fid", ALL_BASIC)
def test_value_at_optimum(orc, fid, dim):
    p = orc.basic(fid, dim, 0)
    f = p(p.shift())[0]
    want = F_OPT + (SCHWEFEL_OFFSET_PER_DIM * dim if fid in (15, 16) else 0.0)
    # Schwefel subtracts D terms of about 419 from 418.9829 D: rounding of that cancellation
    tol = 1e-12 * max(1.0, abs(want)) + (4e-14 * 419.0 * dim * dim if fid in (15, 16) else 0.0)
    assert abs(f - want) <= tol, (fid, dim, f)


@pytest.mark.parametrize("fid", ALL_BASIC)
def test_lower_bound_on_random_points(orc, fid):
    dim = 30
    p = orc.basic(fid, dim, 1)
    rng = np.random.default_rng(fid)
    x = rng.uniform(-100, 100, size=(4000, dim))
    # points close to the optimum too
    x[:1000] = p.shift()[None, :] + rng.normal(scale=0.05, size=(1000, dim))
    f = p(x)
    bound = F_OPT + (SCHWEFEL_OFFSET_PER_DIM * dim if fid in (15, 16) else 0.0)
    assert np.all(np.isfinite(f))
    assert f.min() >= bound - 1e-9


def test_transform_at_optimum_is_the_offset(orc):
    for fid in ALL_BASIC:
        p = orc.basic(fid, 20, 0)
        z = p.transform(p.shift())
        c = orc.XFORM[fid][1]
        assert np.all(z == c), fid


@pytest.mark.parametrize("fid", [2, 11, 19, 14])
def test_transform_orientation(orc, fid):
    """x = o + (t/s) R^T e_j must give z = t e_j + c: catches a transposed rotation."""
    dim = 31
    p = orc.basic(fid, dim, 5)
    R, o = p.rotation(), p.shift()
    s, c, _ = orc.XFORM[fid]
    for j in (0, 7, 30):
        t = 1.75
        x = o + (t / s) * R[j, :]
        z = p.transform(x)
        want = np.full(dim, c)
        want[j] += t
        assert np.abs(z - want).max() < 1e-12


def test_elliptic_end_to_end_axis_values(orc):
    dim = 50
    p = orc.basic(2, dim, 2)
    R, o = p.rotation(), p.shift()
    for j in (0, 1, 25, 49):
        x = o + 3.0 * R[j, :]
        want = 10.0 ** (6.0 * j / (dim - 1)) * 9.0 + F_OPT
        assert abs(p(x)[0] - want) <= 1e-12 * want


def test_rotated_sphere_is_rotation_invariant(orc):
    dim = 100
    p = orc.basic(0, dim, 0)
    rng = np.random.default_rng(0)
    x = rng.uniform(-100, 100, size=(500, dim))
    want = ((x - p.shift()) ** 2).sum(axis=1) + F_OPT
    assert np.abs(p(x) - want).max() <= 1e-13 * want.max()


# ---- closed forms of g on exact z -------------------------------------------------------


def test_sphere_ellipsoid_discus_cigar_axes(orc):
    D = 12
    for j in range(D):
        e = np.zeros(D)
        e[j] = 1.0
        assert orc.g(0, 2 * e) == 4.0
        assert orc.g(1, e) == j + 1
        assert orc.g(3, e) == (1e6 if j == 0 else 1.0)
        assert orc.g(4, e) == (1.0 if j == 0 else 1e6)


def test_elliptic_all_ones(orc):
    D = 10
    want = sum(10.0 ** (6.0 * i / (D - 1)) for i in range(D))
    assert abs(orc.g(2, np.ones(D)) - want) < 1e-9
    assert abs(orc.g(2, np.eye(D)[D - 1]) - 1e6) < 1e-9


def test_powers_and_sharp_valley(orc):
    D = 5
    assert orc.g(5, np.eye(D)[0]) == 1.0
    assert abs(orc.g(5, 2.0 * np.eye(D)[D - 1]) - 8.0) < 1e-14  # |2|^6 = 64
    assert orc.g(6, 3.0 * np.eye(D)[0]) == 9.0
    z = np.zeros(D)
    z[1], z[2] = 3.0, 4.0
    assert abs(orc.g(6, z) - 500.0) < 1e-12


def test_step_plateaus(orc):
    assert orc.g(7, np.array([0.49, -0.5, 1.49, -1.51])) == 0 + 0 + 1 + 4
    assert orc.g(7, np.array([0.5, -0.51])) == 1 + 1


def test_weierstrass_zero_on_integer_lattice(orc):
    for z in (np.zeros(4), np.array([1.0, -2.0, 3.0, 0.0])):
        assert abs(orc.g(8, z)) < 1e-9
    # z = 0.5 makes z + 0.5 an integer, so every cosine is 1 (its maximum) while the constant
    # term is -D sum a^k: g = 2 D (2 - 2^-20)
    z = np.full(3, 0.5)
    assert abs(orc.g(8, z) - 2 * 3 * (2.0 - 2.0 ** -20)) < 1e-9


def test_griewank_cos_lattice(orc):
    D = 6
    m = np.array([1, -2, 0, 3, 1, -1], dtype=float)
    z = 2.0 * math.pi * np.sqrt(np.arange(1, D + 1)) * m
    assert abs(orc.g(9, z) - (z ** 2).sum() / 4000.0) < 1e-12
    assert abs(orc.g(9, np.zeros(D))) < 1e-15


def test_rastrigin_integer_and_half_integer(orc):
    k = np.array([1.0, -3.0, 0.0, 2.0, 5.0])
    assert abs(orc.g(11, k) - (k ** 2).sum()) < 1e-12
    assert abs(orc.g(10, k) - (k ** 2).sum()) < 1e-12
    h = k + 0.5
    assert abs(orc.g(11, h) - ((h ** 2) + 20.0).sum()) < 1e-12
    assert abs(orc.g(10, h) - ((h ** 2) + 20.0).sum()) < 1e-12


def test_rosenbrock_closed_forms(orc):
    D = 9
    assert orc.g(14, np.ones(D)) == 0.0
    assert orc.g(14, np.zeros(D)) == D - 1
    assert orc.g(14, -np.ones(D)) == 404.0 * (D - 1)


def test_grie_rosen_and_schaffer_f6_and_f7(orc):
    D = 7
    assert abs(orc.g(13, np.ones(D))) < 1e-15
    assert abs(orc.g(22, np.zeros(D))) < 1e-15
    # Schaffer F6 pair at radius pi/2: (1 - 0.5)/(1 + 0.001 (pi/2)^2)^2 + 0.5 for each of the D pairs
    # when every neighbouring pair has x^2 + y^2 = (pi/2)^2: z alternating (pi/2)/sqrt(2)
    a = (math.pi / 2) / math.sqrt(2.0)
    z = np.full(4, a)
    one = 0.5 / (1 + 0.001 * (math.pi / 2) ** 2) ** 2 + 0.5
    assert abs(orc.g(22, z) - 4 * one) < 1e-12
    assert abs(orc.g(12, np.zeros(D))) < 1e-15
    # F7 with all w_i = 1: ((1 + sin^2(50)) * 1)^2
    z = np.full(5, 1.0 / math.sqrt(2.0))
    assert abs(orc.g(12, z) - (1.0 + math.sin(50.0) ** 2) ** 2) < 1e-12


def test_schwefel_branches_continuous_and_optimum(orc):
    D = 4
    w0 = 420.9687462275036
    assert abs(orc.g(15, np.zeros(D)) - D * SCHWEFEL_OFFSET_PER_DIM) < 1e-10
    for edge in (500.0, -500.0):
        z = np.full(D, edge - w0)
        lo = orc.g(15, np.nextafter(z, z - 1.0))
        hi = orc.g(15, np.nextafter(z, z + 1.0))
        assert abs(lo - hi) < 1e-9
    # the w > 500 branch folds: w = 500 + t behaves like w = 500 - t less the penalty t^2/(10000 D)
    t = 37.0
    zf = np.full(D, 500.0 + t - w0)
    zm = np.full(D, 500.0 - t - w0)
    assert abs(orc.g(15, zf) - (orc.g(15, zm) + D * t * t / (10000.0 * D))) < 1e-9


def test_katsuura_dyadic(orc):
    D = 3
    assert orc.g(17, np.zeros(D)) == 0.0
    assert abs(orc.g(17, np.full(D, 0.5))) < 1e-15
    ex = 10.0 / D ** 1.2
    want = 10.0 / D ** 2 * (np.prod([(1 + i * 0.25) ** ex for i in range(1, D + 1)]) - 1.0)
    assert abs(orc.g(17, np.full(D, 0.25)) - want) < 1e-13


def test_lunacek_funnels(orc):
    D = 6
    assert abs(orc.g(18, np.full(D, 2.5))) < 1e-12
    assert abs(orc.g(18, np.full(D, -2.5)) - D) < 1e-12


def test_ackley_closed_forms(orc):
    D = 8
    assert abs(orc.g(19, np.zeros(D))) < 1e-14
    s = np.array([1, -1, 1, 1, -1, -1, 1, -1], dtype=float)
    assert abs(orc.g(19, s) - 3.625384938440362) < 1e-13
    assert abs(orc.g(19, np.full(D, 0.5)) - 4.253654026568412) < 1e-13


def test_happycat_hgbat_optimum_and_values(orc):
    D = 5
    assert abs(orc.g(20, -np.ones(D))) < 1e-15
    assert abs(orc.g(21, -np.ones(D))) < 1e-15
    z = np.zeros(D)  # sum z^2 = 0, sum z = 0
    assert abs(orc.g(20, z) - (D ** 0.25 + 0.5)) < 1e-14
    assert abs(orc.g(21, z) - 0.5) < 1e-15


# ---- D = 2 brute force --------------------------------------------------------------------

UNIMODAL = [0, 1, 2, 3, 4, 5, 6]


@pytest.mark.parametrize("fid", ALL_BASIC)
def test_d2_grid_minimum(orc, fid):
    p = orc.basic(fid, 2, 11)
    o = p.shift()
    g = np.linspace(-100.0, 100.0, 801)
    X, Y = np.meshgrid(g, g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    f = p(pts, threads=4)
    bound = F_OPT + (2 * SCHWEFEL_OFFSET_PER_DIM if fid in (15, 16) else 0.0)
    assert f.min() >= bound - 1e-9
    k = int(np.argmin(f))
    # refine around the grid argmin
    c = pts[k]
    h = g[1] - g[0]
    r = np.linspace(-h, h, 201)
    RX, RY = np.meshgrid(c[0] + r, c[1] + r, indexing="ij")
    fr = p(np.stack([RX.ravel(), RY.ravel()], axis=1))
    assert fr.min() >= bound - 1e-9
    if fid in UNIMODAL or fid in (15, 16):
        best = np.stack([RX.ravel(), RY.ravel()], axis=1)[int(np.argmin(fr))]
        assert np.abs(best - o).max() <= h, (fid, best, o)
