"""Pins for the oracle's problem generator (General Setup, Sec. 1.2).

Each check compares the oracle with something other than itself: the published SplitMix64
test vectors, distribution tests from scipy, the orthogonality the paper requires, and
numpy's LAPACK QR (a different factorisation algorithm with the same unique result).
"""
import numpy as np
import pytest
from scipy import stats

M64 = (1 << 64) - 1


def test_splitmix64_published_vectors(orc):
    # SplitMix64 started from state 0 yields these first outputs (the values commonly used
    # to validate implementations of the Steele-Lea-Flood generator).
    assert orc.splitmix64_from_state(0, 0) == 0xE220A8397B1DCDAF
    assert orc.splitmix64_from_state(0, 1) == 0x6E789E6AA1B965F4
    assert orc.splitmix64_from_state(0, 2) == 0x06C45D188009454F


def test_streams_independent_and_uniform(orc):
    a = orc.stream_u64(0, 100, 11 << 8, 0, 20000)
    b = orc.stream_u64(0, 100, 11 << 8, 1, 20000)
    c = orc.stream_u64(1, 100, 11 << 8, 0, 20000)
    assert len(set(a.tolist()) & set(b.tolist())) == 0
    assert len(set(a.tolist()) & set(c.tolist())) == 0
    u = (a >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_normals_are_standard_normal(orc):
    z = orc.stream_normal(7, 30, 3 << 8, 2, 200000)
    assert abs(z.mean()) < 0.01
    assert abs(z.std() - 1.0) < 0.01
    assert stats.kstest(z, "norm").pvalue > 1e-3


@pytest.mark.parametrize("dim", [2, 3, 4, 10, 30, 50, 100, 1000])
def test_rotation_orthonormal_and_block_structure(orc, dim):
    p = orc.basic(11, dim, 0)
    R = p.rotation()
    assert np.abs(R.T @ R - np.eye(dim)).max() <= 1e-13
    assert np.abs(R @ R.T - np.eye(dim)).max() <= 1e-13
    # groups = connected components of the nonzero pattern; sizes floor(D/3) (+1 for the first D mod 3)
    nz = R != 0.0
    seen = np.zeros(dim, bool)
    sizes = []
    for s in range(dim):
        if seen[s]:
            continue
        comp, stack = set(), [s]
        while stack:
            i = stack.pop()
            if i in comp:
                continue
            comp.add(i)
            stack.extend(np.nonzero(nz[i] | nz[:, i])[0].tolist())
        for i in comp:
            seen[i] = True
        sizes.append(len(comp))
        idx = sorted(comp)
        # dense inside the group
        assert nz[np.ix_(idx, idx)].all() or len(comp) == 1
    want = sorted(dim // 3 + (1 if k < dim % 3 else 0) for k in range(3) if dim // 3 + (1 if k < dim % 3 else 0) > 0)
    assert sorted(sizes) == want


def _fisher_yates(u64, dim):
    perm = list(range(dim))
    k = 0
    for i in range(dim - 1, 0, -1):
        j = int(u64[k]) % (i + 1)
        k += 1
        perm[i], perm[j] = perm[j], perm[i]
    return perm


@pytest.mark.parametrize("fid,dim", [(11, 10), (2, 31), (19, 100)])
def test_rotation_blocks_equal_lapack_qr_of_the_normal_draws(orc, fid, dim):
    """Each block is the Q of a QR with positive diagonal of the block's N(0,1) draws."""
    key = fid << 8
    perm = _fisher_yates(orc.stream_u64(0, dim, key, 1, dim), dim)
    sizes = [dim // 3 + (1 if k < dim % 3 else 0) for k in range(3)]
    total = sum(n * n for n in sizes)
    normals = orc.stream_normal(0, dim, key, 2, total)
    R = orc.basic(fid, dim, 0).rotation()
    off, noff = 0, 0
    for n in sizes:
        A = normals[noff:noff + n * n].reshape(n, n)
        Q, Rf = np.linalg.qr(A)
        Q = Q * np.sign(np.diag(Rf))[None, :]
        S = perm[off:off + n]
        assert np.abs(R[np.ix_(S, S)] - Q).max() < 1e-12
        off += n
        noff += n * n


def test_shift_in_range_and_uniform(orc):
    o = orc.basic(0, 1000, 3).shift()
    assert o.min() >= -70.0 and o.max() < 70.0
    assert stats.kstest((o + 70.0) / 140.0, "uniform").pvalue > 1e-3


def test_cgs2_matches_lapack_on_a_334_block(orc):
    rng = np.random.default_rng(0)
    A = rng.standard_normal((334, 334))
    Q = orc.orthonormalise(A)
    assert np.abs(Q.T @ Q - np.eye(334)).max() <= 1e-13
    Ql, Rl = np.linalg.qr(A)
    Ql = Ql * np.sign(np.diag(Rl))[None, :]
    assert np.abs(Q - Ql).max() < 1e-10


def test_problems_differ_per_function_and_dimension(orc):
    a = orc.basic(2, 30, 0).rotation()
    b = orc.basic(9, 30, 0).rotation()
    assert np.abs(a - b).max() > 0.1
    assert np.abs(orc.basic(2, 30, 0).shift() - orc.basic(2, 30, 1).shift()).max() > 1.0
