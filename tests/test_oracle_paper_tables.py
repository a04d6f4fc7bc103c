"""Pins of the oracle's transcribed constants against the values the paper prints.

Fixtures (each row cites its section):
- tests/golden/paper_transforms.txt: s, c and the rotation flag of every Tab. 1 basic function,
  read off the "where" clause of Secs. 3-4;
- tests/golden/paper_hybrids.txt: N, p and the component ids of Hybrid Functions 1-6 (Sec. 5);
- tests/golden/paper_compositions.txt: N, sigma, lambda, bias and the component ids of
  Composition Functions 1-8 (Sec. 6).

Each table is checked twice: element by element against the oracle's own table, and through
behaviour that only the right value produces -- the transform of a displaced optimum
(z = t s R e_j + c, Sec. 1.2), hybrid group sizes (Eq. (numbers)) and whole hybrid and
composition values re-assembled here from the fixture's parameters and the separately pinned
formulas g (Eqs. (hybrid), (composition), (weight)).  A single mistyped s, c, p, sigma, lambda
or G id in the oracle fails at least one of them.
"""
import math
import os

import numpy as np
import pytest

F_OPT = 100.0
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            yield line.split()


def _floats(s):
    return [float(v) for v in s.split(",")]


def _ints(s):
    return [int(v) for v in s.split(",")]


TRANSFORMS = {int(r[0]): (float(r[1]), float(r[2]), bool(int(r[3]))) for r in _rows("paper_transforms.txt")}
HYBRIDS = {int(r[0]): (int(r[1]), _floats(r[2]), _ints(r[3])) for r in _rows("paper_hybrids.txt")}
COMPOSITIONS = {int(r[0]): (int(r[1]), _floats(r[2]), _floats(r[3]), _floats(r[4]), _ints(r[5]))
                for r in _rows("paper_compositions.txt")}


def test_fixtures_are_complete():
    assert sorted(TRANSFORMS) == list(range(23))
    assert sorted(HYBRIDS) == list(range(23, 29))
    assert sorted(COMPOSITIONS) == list(range(29, 37))
    for n, p, g in HYBRIDS.values():
        assert len(p) == len(g) == n
        assert abs(sum(p) - 1.0) < 1e-12
    for n, sig, lam, bias, g in COMPOSITIONS.values():
        assert len(sig) == len(lam) == len(bias) == len(g) == n


# ---- basic transforms (Secs. 3-4) --------------------------------------------------------

@pytest.mark.parametrize("fid", range(23))
def test_transform_table_matches_paper(orc, fid):
    assert orc.table_xform(fid) == TRANSFORMS[fid]
    p = orc.basic(fid, 12, 0)
    assert p.basic_params() == (fid,) + TRANSFORMS[fid]


@pytest.mark.parametrize("fid", range(23))
def test_displaced_optimum_gives_scaled_rotation_column(orc, fid):
    """x = o + t e_j gives z = t s R[:, j] + c (Sec. 1.2 with the section's s and c): pins s, c
    and the rotation flag through the transform itself, not through any table."""
    s, c, rotated = TRANSFORMS[fid]
    dim = 17
    p = orc.basic(fid, dim, 3)
    o, R = p.shift(), p.rotation()
    if not rotated:
        assert np.array_equal(R, np.eye(dim))
    else:
        assert np.count_nonzero(np.abs(R - np.eye(dim)) > 1e-3) > dim
    for j in (0, 5, dim - 1):
        for t in (1.0, -3.5):
            x = o.copy()
            x[j] += t
            z = p.transform(x)
            want = t * s * R[:, j] + c
            assert np.abs(z - want).max() <= 1e-12 * max(1.0, abs(t * s)) + 1e-13, (fid, j, t)


# ---- hybrids (Sec. 5) --------------------------------------------------------------------

@pytest.mark.parametrize("fid", range(23, 29))
def test_hybrid_table_matches_paper(orc, fid):
    n, p, g = HYBRIDS[fid]
    assert orc.table_hybrid(fid) == (p, g)
    prob = orc.fid_problem(fid, 40, 0)
    assert prob.group_bases() == g
    assert prob.ncomp() == n


def _group_sizes(p, dim):
    """Eq. (numbers): n_i = ceil(p_i D) for i < N, the rest for the last."""
    sizes = [math.ceil(pi * dim) for pi in p[:-1]]
    return sizes + [dim - sum(sizes)]


def _hybrid_value(orc, prob, g, x):
    """Eq. (hybrid) re-assembled from the fixture's ids and transforms: y = x - o, group i takes
    the next n_i entries of y permuted by S, z^i = R_i (s_i y^i) + c_i, F = sum g_i(z^i) + f_opt."""
    perm, sizes, blocks = prob.hybrid_parts()
    y = x - prob.shift()
    F, off = 0.0, 0
    for i, n in enumerate(sizes):
        s, c, _ = TRANSFORMS[g[i]]
        v = s * y[perm[off:off + n]]
        F += orc.g(g[i], blocks[i] @ v + c)
        off += n
    return F + F_OPT


@pytest.mark.parametrize("dim", [10, 30, 100])
@pytest.mark.parametrize("fid", range(23, 29))
def test_hybrid_structure_and_value(orc, fid, dim):
    n, p, g = HYBRIDS[fid]
    prob = orc.fid_problem(fid, dim, 1)
    perm, sizes, _ = prob.hybrid_parts()
    assert list(sizes) == _group_sizes(p, dim)
    assert sorted(perm) == list(range(dim))
    rng = np.random.default_rng(fid * 1000 + dim)
    for x in rng.uniform(-100, 100, size=(4, dim)):
        want = _hybrid_value(orc, prob, g, x)
        got = prob(x[None, :])[0]
        assert abs(got - want) <= 1e-12 * max(1.0, abs(want)), (fid, dim, got, want)


# ---- compositions (Sec. 6) ---------------------------------------------------------------

@pytest.mark.parametrize("fid", range(29, 37))
def test_composition_table_matches_paper(orc, fid):
    n, sig, lam, bias, g = COMPOSITIONS[fid]
    assert orc.table_composition(fid) == (sig, lam, g)
    prob = orc.fid_problem(fid, 20, 0)
    assert prob.ncomp() == n
    s_, l_, b_ = prob.blend_params()
    assert list(s_) == sig and list(l_) == lam and list(b_) == bias
    for i in range(n):
        comp = prob.component(i)
        if g[i] >= 23:
            assert comp.group_bases() == HYBRIDS[g[i]][2]
        else:
            assert comp.basic_params() == (g[i],) + TRANSFORMS[g[i]]
        # the third component's optimum sits at the origin (Sec. 6)
        assert (np.count_nonzero(comp.shift()) == 0) == (i == 2), (fid, i)


def _component_value(orc, comp, gid, x):
    """G_i(x) without f_opt: the basic formula under the fixture's transform, or a hybrid."""
    if gid >= 23:
        return _hybrid_value(orc, comp, HYBRIDS[gid][2], x) - F_OPT
    s, c, _ = TRANSFORMS[gid]
    z = comp.rotation() @ (s * (x - comp.shift())) + c
    return orc.g(gid, z)


@pytest.mark.parametrize("fid", range(29, 37))
def test_composition_value_reassembled(orc, fid):
    """Eqs. (composition) and (weight) with the fixture's sigma, lambda, bias and ids:
    w_i = exp(-d_i^2 / (2 D sigma_i^2)) / d_i, omega = w / sum w, F = sum omega_i (lambda_i G_i +
    bias_i) + f_opt.  Points are drawn near each optimum too, where one weight dominates."""
    n, sig, lam, bias, g = COMPOSITIONS[fid]
    dim = 20
    prob = orc.fid_problem(fid, dim, 2)
    rng = np.random.default_rng(fid)
    pts = list(rng.uniform(-100, 100, size=(3, dim)))
    for i in range(n):
        pts.append(prob.component(i).shift() + rng.normal(scale=8.0, size=dim))
    for x in pts:
        d2 = np.array([np.sum((x - prob.component(i).shift()) ** 2) for i in range(n)])
        logw = -0.5 * np.log(d2) - d2 / (2.0 * dim * np.asarray(sig) ** 2)
        w = np.exp(logw - logw.max())
        om = w / w.sum()
        G = np.array([_component_value(orc, prob.component(i), g[i], x) for i in range(n)])
        want = float(np.sum(om * (np.asarray(lam) * G + np.asarray(bias))) + F_OPT)
        got = prob(x[None, :])[0]
        assert abs(got - want) <= 1e-11 * max(1.0, abs(want)), (fid, got, want)
