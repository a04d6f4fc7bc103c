"""Pins for the oracle's differential evolution (the reference of the GPU optimiser).

The oracle's DE is checked against a second implementation of the same specification written
here in plain Python (exact fused multiply-add through rational arithmetic, SplitMix64 from its
published definition, whose first outputs from state 0 are the published test vectors), on
tiny runs, bit for bit; and against the invariants of greedy selection: no value ever
increases, every stored value is the formula's value of the stored vector, vectors stay in the
search box, and with CR = 0 a trial differs from its target in exactly one variable.
"""
from fractions import Fraction

import numpy as np
import pytest

M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def mix64(z):
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def draw(seed, k):
    return mix64((seed + (k + 1) * GAMMA) & M64)


def fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def test_draw_is_splitmix64():
    assert draw(0, 0) == 0xE220A8397B1DCDAF
    assert draw(0, 1) == 0x6E789E6AA1B965F4
    assert draw(0, 2) == 0x06C45D188009454F


def de_python(f, pop, fit, F, CR, seed, gen0, gens):
    """DE/rand/1/bin, one generation after the other, written from the specification."""
    pop, fit = pop.copy(), fit.copy()
    n, D = pop.shape
    for g in range(gen0, gen0 + gens):
        trial = pop.copy()
        for i in range(n):
            base = (g * n + i) * (D + 4)
            allowed = [a for a in range(n) if a != i]
            r = []
            for t in range(3):
                r.append(allowed.pop(draw(seed, base + t) % len(allowed)))
            jr = draw(seed, base + 3) % D
            for j in range(D):
                u = (draw(seed, base + 4 + j) >> 11) * 2.0 ** -53
                if u < CR or j == jr:
                    v = fma(F, pop[r[1], j] - pop[r[2], j], pop[r[0], j])
                    trial[i, j] = min(max(v, -100.0), 100.0)
        ft = f(trial)
        take = ft <= fit
        pop[take] = trial[take]
        fit[take] = ft[take]
    return pop, fit


@pytest.mark.parametrize("fid,dim,np_,CR", [(0, 3, 5, 0.9), (11, 4, 6, 0.5), (14, 2, 4, 1.0), (19, 5, 7, 0.0)])
def test_oracle_de_equals_python_de(orc, fid, dim, np_, CR):
    p = orc.basic(fid, dim, 0)
    rng = np.random.default_rng(fid)
    pop = rng.uniform(-100, 100, size=(np_, dim))
    fit = p(pop)
    want_pop, want_fit = de_python(p, pop, fit, 0.7, CR, 12345, 3, 4)
    got_pop, got_fit = pop.copy(), fit.copy()
    p.de_run(got_pop, got_fit, 0.7, CR, 12345, 3, 4)
    assert np.array_equal(got_pop, want_pop)
    assert np.array_equal(got_fit, want_fit)


def test_selection_invariants(orc):
    dim, n = 10, 50
    p = orc.basic(11, dim, 0)
    pop = np.random.default_rng(1).uniform(-100, 100, size=(n, dim))
    fit = p(pop)
    best0 = fit.min()
    prev_fit = fit.copy()
    for g in range(20):
        p.de_run(pop, fit, 0.5, 0.9, 7, g, 1)
        assert np.all(fit <= prev_fit)
        assert np.all(np.abs(pop) <= 100.0)
        assert np.array_equal(fit, p(pop))
        prev_fit = fit.copy()
    assert fit.min() < best0


def test_cr_zero_changes_one_variable(orc):
    dim, n = 8, 10
    p = orc.basic(0, dim, 0)
    pop0 = np.random.default_rng(2).uniform(-100, 100, size=(n, dim))
    # make every trial win, so the stored vectors are the trials: a constant function is not
    # available, so start from the worst values (huge) the sphere cannot exceed
    pop, fit = pop0.copy(), np.full(n, np.inf)
    p.de_run(pop, fit, 0.5, 0.0, 3, 0, 1)
    changed = (pop != pop0).sum(axis=1)
    assert np.all(changed == 1)
