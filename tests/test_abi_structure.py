"""Problem-structure export through the C ABI (curob_generate_* host-only forms, no GPU),
compared with the oracle's independent generator part by part:

- hybrids (Sec. 5, Eq. (hybrid)): shift o, permutation S, group sizes n_i (Eq. (numbers)), the
  per-group rotations R_i, and each group's formula id, scale and offset;
- compositions (Sec. 6, Eqs. (composition), (weight)): sigma_i, lambda_i, bias_i and every
  component's o^i and rotation (the third at the origin), hybrid components included.

o and S come from the same published generator on both sides and must be bit-identical; the
rotations are orthonormalised differently (Householder vs Gram-Schmidt) and agree to 1e-13.
Formula ids and transforms are also checked against the paper fixtures in tests/golden/.
"""
import ctypes
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            yield line.split()


TRANSFORMS = {int(r[0]): (float(r[1]), float(r[2])) for r in _rows("paper_transforms.txt")}
HYBRID_G = {int(r[0]): [int(v) for v in r[3].split(",")] for r in _rows("paper_hybrids.txt")}
COMPS = {int(r[0]): ([float(v) for v in r[2].split(",")], [float(v) for v in r[3].split(",")],
                     [float(v) for v in r[4].split(",")], [int(v) for v in r[5].split(",")])
         for r in _rows("paper_compositions.txt")}


@pytest.fixture(scope="module")
def curob():
    import paper_1407_7737_amd as c
    return c


def _check_hybrid(st, ref, gids):
    """Library structure st against oracle hybrid ref with formula ids gids."""
    perm, sizes, blocks = ref.hybrid_parts()
    assert st["type"] == "hybrid"
    assert np.array_equal(st["o"], ref.shift())
    assert np.array_equal(st["perm"], perm)
    assert np.array_equal(st["sizes"], sizes)
    for a, b in zip(st["blocks"], blocks):
        assert np.abs(a - b).max() <= 1e-13
    assert list(st["bases"]) == gids
    assert [(s, c) for s, c in zip(st["scale"], st["offset"])] == [TRANSFORMS[g] for g in gids]


def _dense(st, dim):
    """Dense rotation of a basic part from its blocks (R[S[a]][S[b]] = Q[a][b])."""
    if st["count"] == 0:
        return np.eye(dim)
    R = np.zeros((dim, dim))
    off = 0
    for n, Q in zip(st["sizes"], st["blocks"]):
        idx = st["perm"][off:off + n]
        R[np.ix_(idx, idx)] = Q
        off += n
    return R


@pytest.mark.parametrize("dim", [10, 30, 100])
@pytest.mark.parametrize("fid", range(23, 29))
def test_hybrid_structure_matches_oracle(curob, orc, fid, dim):
    st = curob.generate_structure(fid, dim, 0)
    assert st["count"] == len(HYBRID_G[fid])
    _check_hybrid(st, orc.fid_problem(fid, dim, 0), HYBRID_G[fid])


@pytest.mark.parametrize("dim", [10, 30])
@pytest.mark.parametrize("fid", range(29, 37))
def test_composition_structure_matches_oracle(curob, orc, fid, dim):
    sig, lam, bias, gids = COMPS[fid]
    top = curob.generate_structure(fid, dim, 4)
    assert top["type"] == "composition" and top["count"] == len(gids)
    s, l, b = curob.generate_composition(fid, dim, 4)
    assert list(s) == sig and list(l) == lam and list(b) == bias
    ref = orc.fid_problem(fid, dim, 4)
    for i, g in enumerate(gids):
        st = curob.generate_structure(fid, dim, 4, comp=i)
        rc = ref.component(i)
        if g >= 23:
            _check_hybrid(st, rc, HYBRID_G[g])
        else:
            assert st["type"] == "basic"
            assert list(st["bases"]) == [g]
            assert (st["scale"][0], st["offset"][0]) == TRANSFORMS[g]
            assert np.array_equal(st["o"], rc.shift())
            assert np.abs(_dense(st, dim) - rc.rotation()).max() <= 1e-13
        # the third component's optimum sits at the origin (Sec. 6)
        assert (np.count_nonzero(st["o"]) == 0) == (i == 2)


@pytest.mark.parametrize("fid,dim", [(0, 2), (11, 31), (10, 20), (16, 100), (14, 200)])
def test_basic_structure_matches_oracle(curob, orc, fid, dim):
    st = curob.generate_structure(fid, dim, 9)
    ref = orc.basic(fid, dim, 9)
    assert st["type"] == "basic"
    assert list(st["bases"]) == [fid] and (st["scale"][0], st["offset"][0]) == TRANSFORMS[fid]
    assert np.array_equal(st["o"], ref.shift())
    assert np.abs(_dense(st, dim) - ref.rotation()).max() <= 1e-13
    if st["count"]:
        # three near-equal groups (Sec. 1.2)
        assert sorted(st["sizes"]) == sorted(dim // 3 + (k < dim % 3) for k in range(3) if dim // 3 + (k < dim % 3))


def test_structure_export_errors(curob):
    lib = curob.lib
    i = ctypes.c_int()
    assert lib.curob_generate_info(37, 10, 0, -1, ctypes.byref(i), None, None) == curob.CUROB_E_FID
    assert lib.curob_generate_info(23, 9, 0, -1, ctypes.byref(i), None, None) == curob.CUROB_E_ARG
    assert lib.curob_generate_info(29, 10, 0, 5, ctypes.byref(i), None, None) == curob.CUROB_E_ARG
    assert lib.curob_generate_info(11, 10, 0, 0, ctypes.byref(i), None, None) == curob.CUROB_E_ARG
    # a composition as a whole has no single structure
    assert lib.curob_generate_structure(29, 10, 0, -1, None, None, None, None, None, None, None) == curob.CUROB_E_ARG
    assert lib.curob_generate_composition(11, 10, 0, None, None, None) == curob.CUROB_E_ARG
    assert lib.curob_get_info(11, -1, None, None, None) == curob.CUROB_E_STATE
    assert lib.curob_get_dim(None, None) == curob.CUROB_E_STATE


def test_binding_rejects_wrong_row_width(curob):
    """Rows must have the initialised dimension (checked before any device call)."""
    import numpy as np
    old = curob._dim
    curob._dim = 12
    try:
        with pytest.raises(ValueError):
            curob.h_func_evaluatef(0, np.zeros((3, 11), dtype=np.float32))
        with pytest.raises(ValueError):
            curob.get_problem(0, 11)
    finally:
        curob._dim = old


def test_undefined_hybrids_match_the_oracle():
    """Where the group sizes of Sec. 5 (n_i = ceil(p_i D), the last group the remainder) give a
    group fewer variables than its formula needs, the hybrid (and a composition built on it) is
    undefined.  The library's host generator and the oracle's refuse exactly the same (id, D)
    pairs over D = 2..200: every hybrid below 10, hybrids 27 and 28 and composition 36 at 11,
    hybrid 27 and composition 36 at 12, nothing else."""
    import oracle
    import paper_1407_7737_amd as curob
    lib = curob.lib
    kind = ctypes.c_int()
    refused_lib, refused_orc = set(), set()
    for dim in range(2, 201):
        for fid in (23, 24, 25, 26, 27, 28, 35, 36):
            if lib.curob_generate_info(fid, dim, 0, -1, ctypes.byref(kind), None, None) != curob.CUROB_OK:
                refused_lib.add((fid, dim))
            try:
                oracle.fid_problem(fid, dim, 0)
            except ValueError:
                refused_orc.add((fid, dim))
    expected = {(f, d) for f in (23, 24, 25, 26, 27, 28, 35, 36) for d in range(2, 10)}
    expected |= {(27, 11), (28, 11), (36, 11), (27, 12), (36, 12)}
    assert refused_lib == expected, sorted(refused_lib ^ expected)
    assert refused_orc == expected, sorted(refused_orc ^ expected)
