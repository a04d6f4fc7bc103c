"""Pins for the oracle's hybrid (Sec. 5) and composition (Sec. 6) constructions."""
import math

import numpy as np
import pytest

F_OPT = 100.0
STAR = [0, 2, 9, 10, 11, 14, 16, 19]


def test_hybrid_group_sizes_follow_the_ceiling_rule(orc):
    # n_i = ceil(p_i D) for i < N, the last group takes the rest (Eq. (numbers))
    for dim, p, want in [(10, [0.3, 0.3, 0.4], [3, 3, 4]),
                         (100, [0.1, 0.2, 0.2, 0.2, 0.3], [10, 20, 20, 20, 30]),
                         (1000, [0.2, 0.2, 0.3, 0.3], [200, 200, 300, 300]),
                         (37, [0.25, 0.3, 0.45], [10, 12, 15])]:
        h = orc.hybrid(200, dim, 0, [2] * len(p), p)
        perm, sizes, blocks = h.hybrid_parts()
        assert sizes.tolist() == want
        assert sorted(perm.tolist()) == list(range(dim))
        for B in blocks:
            assert np.abs(B.T @ B - np.eye(B.shape[0])).max() <= 1e-13


def test_hybrid_group_size_rules(orc):
    # an elliptic group of one variable has the exponent 0/0: rejected
    with pytest.raises(ValueError):
        orc.hybrid(201, 10, 0, [2, 2, 2], [0.05, 0.9, 0.05])
    # Schaffer F6 and Katsuura are defined on one variable (Hybrid 5 and 6 at D = 10)
    h = orc.hybrid(201, 10, 0, [22, 17, 2], [0.1, 0.1, 0.8])
    assert h.hybrid_parts()[1].tolist() == [1, 1, 8]
    assert abs(h(h.shift())[0] - 100.0) < 1e-12
    for fid in (27, 28):
        p = orc.fid_problem(fid, 10, 0)
        assert p(p.shift())[0] >= 100.0


def test_hybrid_of_spheres_is_the_shifted_sphere(orc):
    """Sphere groups: sum ||R_i z^i||^2 = ||x - o||^2 whatever S and R_i are."""
    dim = 60
    h = orc.hybrid(202, dim, 3, [0, 0, 0, 0], [0.2, 0.3, 0.1, 0.4])
    rng = np.random.default_rng(1)
    x = rng.uniform(-100, 100, size=(200, dim))
    want = ((x - h.shift()) ** 2).sum(axis=1) + F_OPT
    assert np.abs(h(x) - want).max() <= 1e-13 * want.max()


@pytest.mark.parametrize("bases", [[16, 11, 2], [9, 14, 19, 10, 0], [21, 3, 13, 10], [17, 20, 13, 15, 19]])
def test_hybrid_optimum(orc, bases):
    dim = 50
    p = [1.0 / len(bases)] * len(bases)
    h = orc.hybrid(203, dim, 0, bases, p)
    _, sizes, _ = h.hybrid_parts()
    f = h(h.shift())[0]
    # Schwefel-based groups keep the per-dimension offset of their n_i variables
    off = sum(n * (418.9829 - 420.9687462275036 * math.sin(math.sqrt(420.9687462275036)))
              for b, n in zip(bases, sizes) if b in (15, 16))
    assert abs(f - (F_OPT + off)) <= 1e-9


def test_hybrid_single_group_separable_function_ignores_permutation(orc):
    """One unrotated-style check: a single-group hybrid of the elliptic function has value
    g(R_1 y[S]) and must equal the elliptic closed form along the rotated axes."""
    dim = 20
    h = orc.hybrid(204, dim, 4, [2], [1.0])
    perm, sizes, blocks = h.hybrid_parts()
    R1 = blocks[0]
    o = h.shift()
    for j in (0, 9, 19):
        # choose x so that R_1 (x - o)[S] = 2 e_j
        v = 2.0 * R1[j, :]
        x = o.copy()
        x[perm] += v
        want = 10.0 ** (6.0 * j / (dim - 1)) * 4.0 + F_OPT
        assert abs(h(x)[0] - want) <= 1e-12 * want


def test_hybrid_lower_bound(orc):
    dim = 40
    h = orc.hybrid(205, dim, 9, [16, 11, 2, 19], [0.3, 0.2, 0.3, 0.2])
    rng = np.random.default_rng(2)
    x = rng.uniform(-100, 100, size=(3000, dim))
    assert h(x).min() >= F_OPT


def _comp(orc, dim, bases, sigma, lam, bias, pid=300, seed=0):
    return orc.composition(pid, dim, seed, bases, sigma, lam, bias)


def test_composition_one_hot_at_each_optimum(orc):
    dim = 30
    bias = [100.0 * i for i in range(8)]
    c = _comp(orc, dim, STAR, [10, 15, 20, 25, 30, 35, 40, 50], [1e-6, 1e-3, 0.1, 1, 0.5, 1e-2, 1e-4, 0.3], bias)
    for k in range(8):
        ok = c.shift(k)
        f = c(ok)[0]
        # component k's own value at its optimum is 0 (Schwefel: 30 * 1.27e-5 times lambda = 1e-4)
        assert abs(f - (bias[k] + F_OPT)) < 1e-7, (k, f)


def test_composition_weights_sum_to_one(orc):
    """With lambda = 0 and equal biases B, F = B sum(omega) + f_opt = B + f_opt."""
    dim = 25
    c = _comp(orc, dim, STAR, [10, 20, 30, 40, 50, 12, 14, 16], [0.0] * 8, [42.0] * 8)
    rng = np.random.default_rng(3)
    x = rng.uniform(-100, 100, size=(500, dim))
    assert np.abs(c(x) - (42.0 + F_OPT)).max() < 1e-12


def test_composition_two_components_weight_closed_form(orc):
    """lambda = 0, biases (0, 1): F - f_opt is omega_2 itself.  At the midpoint of the two
    optima d_1 = d_2 = d, so omega_2 = 1/(1 + exp(d^2/(2D) (1/sigma_2^2 - 1/sigma_1^2)))."""
    dim = 12
    s1, s2 = 10.0, 30.0
    c = _comp(orc, dim, [0, 2], [s1, s2], [0.0, 0.0], [0.0, 1.0], pid=301)
    o1, o2 = c.shift(0), c.shift(1)
    mid = 0.5 * (o1 + o2)
    d2 = ((mid - o1) ** 2).sum()
    want = 1.0 / (1.0 + math.exp(d2 / (2 * dim) * (1 / s2 ** 2 - 1 / s1 ** 2)))
    assert abs(c(mid)[0] - F_OPT - want) < 1e-13
    # equal sigmas: exactly one half at the midpoint
    c2 = _comp(orc, dim, [0, 2], [20.0, 20.0], [0.0, 0.0], [0.0, 1.0], pid=301)
    assert abs(c2(mid)[0] - F_OPT - 0.5) < 1e-15
    # moving toward o2 raises omega_2 monotonically to 1
    ts = np.linspace(0.0, 1.0, 41)
    vals = c(np.array([o1 + t * (o2 - o1) for t in ts]))[1:-1] - F_OPT
    assert np.all(np.diff(vals) > 0)
    # and a point near o1 is dominated by component 1, scaled as 1/d times the Gaussian factor
    x = o1 + 1e-3 * (o2 - o1)
    assert c(x)[0] - F_OPT < 1e-3


def test_composition_single_sphere_component(orc):
    dim = 40
    c = _comp(orc, dim, [0], [20.0], [0.7], [5.0], pid=302)
    rng = np.random.default_rng(4)
    x = rng.uniform(-100, 100, size=(100, dim))
    want = 0.7 * ((x - c.shift(0)) ** 2).sum(axis=1) + 5.0 + F_OPT
    assert np.abs(c(x) - want).max() <= 1e-13 * want.max()


def test_composition_is_a_convex_combination(orc):
    dim = 20
    lam = [1e-6, 1e-3, 0.1, 1, 0.5, 1e-2, 1e-4, 0.3]
    bias = [100.0 * i for i in range(8)]
    c = _comp(orc, dim, STAR, [10, 15, 20, 25, 30, 35, 40, 50], lam, bias, pid=303)
    rng = np.random.default_rng(5)
    x = rng.uniform(-100, 100, size=(300, dim))
    F = c(x) - F_OPT
    assert np.all(F >= 0.0)
    # never above the largest component term lambda_i G_i + bias_i; sphere-like upper bound check
    assert np.all(F <= 700.0 + max(lam) * 1e12)


@pytest.mark.parametrize("fid", list(range(23, 37)))
def test_paper_tables_build_and_hit_their_optima(orc, fid):
    dim = 30
    p = orc.fid_problem(fid, dim, 0)
    rng = np.random.default_rng(fid)
    x = rng.uniform(-100, 100, size=(200, dim))
    f = p(x)
    assert np.all(np.isfinite(f)) and f.min() >= F_OPT - 1e-9
    if fid >= 29:
        # third optimum at the origin (the trap of Sec. 6): F(0) = lambda_3 G_3(0) + bias_3 + f_opt,
        # where G_3(0) is 0 except for Schwefel-based components (n * 1.27e-5, lambda <= 10)
        tol = 10.0 * dim * 1.3e-5
        assert abs(p(np.zeros(dim))[0] - (200.0 + F_OPT)) < tol
        assert abs(p(p.shift(0))[0] - F_OPT) < tol
        if fid == 29:  # no Schwefel-based component: the optima are exact
            assert abs(p(np.zeros(dim))[0] - (200.0 + F_OPT)) < 1e-9


def test_paper_hybrids_need_dimension_ten(orc):
    with pytest.raises(ValueError):
        orc.fid_problem(23, 9, 0)
