"""GPU parity: every evaluation path against the FP64 oracle on the same seeded inputs.

Bars (stated for the whole suite): FP64 path |f - f_oracle| <= 1e-10 max(1, |f_oracle|);
FP32 paths |f - f_oracle| <= 1e-4 max(1, |f_oracle|), FP32 inputs widened exactly for the
oracle.  The default split mode and the plain FP32 mode meet the FP32 bar on every formula;
the pure three-product split mode meets it on the formulas it is chosen for by default.
Step and the rotated/unrotated Schwefel g1 are discontinuous (plateau edges; jumps at
|w| = 1000, 1500, ...): rows whose oracle z lies within the FP32 path's rounding of such an
edge can land on either side, so those rows (a small fraction) are checked for finiteness
and excluded from the bound.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-4
SEED = 0
# formulas the default split mode evaluates with six BF16 products (Rosenbrock below D = 10,
# elliptic below D = 50)
SIX_PRODUCTS = {3, 7, 8, 12, 13, 16, 17}


def six(fid, dim):
    return fid in SIX_PRODUCTS or (fid in (4, 14) and dim < 10) or (fid == 2 and dim < 50)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    import paper_1407_7737_amd as c
    import oracle
    state = {"dim": None}

    def use(dim, maxc=1 << 18, seed=SEED):
        if state["dim"] != (dim, maxc, seed):
            if state["dim"] is not None:
                c.dispose()
            c.initialize(dim, maxc, seed)
            state["dim"] = (dim, maxc, seed)

    yield c, oracle, torch, use
    if state["dim"] is not None:
        c.dispose()


def rel_err(f, ref):
    f = np.asarray(f, dtype=np.float64)
    return np.abs(f - ref) / np.maximum(1.0, np.abs(ref))


def oracle_z(orc, fid, p, x):
    """z = R(s(x - o)) + c of the oracle's problem, and y = s(x - o), per row."""
    s, c, _ = orc.XFORM[fid]
    y = s * (x - p.shift()[None, :])
    return y @ p.rotation().T + c, y


def check32(orc, fid, p, x32w, f, ref, tag):
    """FP32 bar, with the discontinuous formulas handled as the module docstring says."""
    e = rel_err(f, ref)
    assert np.all(np.isfinite(f)), (tag, fid)
    if fid == 7:
        # Step: z within the FP32 rotation's rounding of a plateau edge may round either way.
        # Most rows meet the bar; every row is within two plateau jumps (2|k| + 1 each).
        z, _ = oracle_z(orc, fid, p, x32w)
        jump = 2.0 * (2.0 * np.abs(z).max(axis=1) + 3.0)
        assert (e <= TOL32).mean() >= 0.9, (tag, fid, (e <= TOL32).mean())
        assert np.all(np.abs(np.asarray(f, np.float64) - ref) <= jump + TOL32 * np.abs(ref)), (tag, fid)
        return float(np.median(e))
    if fid in (15, 16):
        # modified Schwefel g1 jumps where |w| = |z + 420.97| crosses 1000, 1500, ...; rows with
        # a component within a generous FP32 rotation error (64 ulp of |y|) of a jump are excluded
        z, y = oracle_z(orc, fid, p, x32w)
        w = np.abs(z + 420.9687462275036)
        d = np.where(w >= 750.0, np.abs(w - 500.0 * np.round(w / 500.0)), np.inf)
        delta = 64.0 * 2.0 ** -24 * (1.0 + np.linalg.norm(y, axis=1, keepdims=True))
        edge = (d < delta).any(axis=1)
        assert edge.mean() <= 0.02, (tag, fid, edge.mean())
        e = np.where(edge, 0.0, e)
    assert e.max() <= TOL32, (tag, fid, float(e.max()))
    return float(e.max())


def run_paths(c, torch, fid, x64, modes):
    """FP64 result and FP32 results per mode for the same points (FP32 points = x64 rounded)."""
    x32 = x64.astype(np.float32)
    dx64 = torch.from_numpy(x64).cuda()
    dx32 = torch.from_numpy(x32).cuda()
    f64 = c.func_evaluate(fid, dx64).cpu().numpy()
    out = {}
    for m in modes:
        c.set_mode(m)
        out[m] = c.func_evaluatef(fid, dx32).cpu().numpy()
    c.set_mode(c.MODE_SPLIT)
    torch.cuda.synchronize()
    return x32.astype(np.float64), f64, out


@pytest.mark.parametrize("dim", [2, 3, 10, 17, 30, 50, 64, 100, 128])
def test_all_basic_functions_all_paths(env, dim):
    c, orc, torch, use = env
    use(dim)
    from paper_1407_7737_amd.inputs import population, near
    n = 1000  # 62 full groups of 16 rows and a ragged tail of 8
    modes = [c.MODE_SPLIT, c.MODE_FP32, c.MODE_SPLIT_BF16X3, c.MODE_SPLIT_BF16X6]
    for fid in range(23):
        say(f"[parity] dim={dim} fid={fid} n={n}")
        p = orc.basic(fid, dim, SEED)
        x = population(n, dim, seed=fid)
        x[:100] = near(np.repeat(p.shift()[None, :], 100, axis=0), 0.5, seed=fid)  # small f regime
        x32w, f64, f = run_paths(c, torch, fid, x, modes)
        e64 = rel_err(f64, p(x)).max()
        assert e64 <= TOL64, (fid, dim, e64)
        ref32 = p(x32w)
        check32(orc, fid, p, x32w, f[c.MODE_SPLIT], ref32, "split")
        check32(orc, fid, p, x32w, f[c.MODE_FP32], ref32, "fp32")
        check32(orc, fid, p, x32w, f[c.MODE_SPLIT_BF16X6], ref32, "split-x6")
        if not six(fid, dim):
            check32(orc, fid, p, x32w, f[c.MODE_SPLIT_BF16X3], ref32, "split-x3")
        else:
            assert np.all(np.isfinite(f[c.MODE_SPLIT_BF16X3]))


def test_every_resident_dimension(env):
    """Every dimension the resident kernel takes (2..128): row stride, k- and m-tile counts,
    aligned and unaligned rows, rows loaded straight into LDS or staged through registers.  An
    unrotated formula, a rotated one, one with pair terms and a six-product one, 1000 rows (62
    row groups and a ragged 8; the Schwefel check bounds the share of rows at a jump), every FP32
    mode and FP64, against the oracle."""
    c, orc, torch, use = env
    from paper_1407_7737_amd.inputs import population
    n = 1000
    for dim in range(2, 129):
        use(dim, maxc=n)
        for fid in (0, 11, 14, 16):
            say(f"[every-dim] dim={dim} fid={fid}")
            p = orc.basic(fid, dim, SEED)
            x = population(n, dim, seed=dim)
            modes = [c.MODE_SPLIT, c.MODE_FP32, c.MODE_SPLIT_BF16X6] + ([] if six(fid, dim) else [c.MODE_SPLIT_BF16X3])
            x32w, f64, f = run_paths(c, torch, fid, x, modes)
            assert rel_err(f64, p(x)).max() <= TOL64, (dim, fid)
            ref32 = p(x32w)
            for m in modes:
                check32(orc, fid, p, x32w, f[m], ref32, ("every-dim", dim, m))


@pytest.mark.parametrize("n", [1, 2, 15, 16, 17, 63, 64, 65, 257, 4097])
def test_ragged_row_counts(env, n):
    c, orc, torch, use = env
    use(100)
    from paper_1407_7737_amd.inputs import population
    for fid in (11, 14):
        say(f"[ragged] n={n} fid={fid}")
        p = orc.basic(fid, 100, SEED)
        x = population(n, 100, seed=n)
        x32w, f64, f = run_paths(c, torch, fid, x, [c.MODE_SPLIT, c.MODE_FP32])
        assert f64.shape == (n,) and f[c.MODE_SPLIT].shape == (n,)
        assert rel_err(f64, p(x)).max() <= TOL64
        for m in f:
            assert rel_err(f[m], p(x32w)).max() <= TOL32


@pytest.mark.parametrize("dim", [97, 100, 128])
def test_rows_not_16_byte_aligned(env, dim):
    """Rows that do not start 16-byte aligned (a population one float into its buffer, or
    D not a multiple of 4) take the resident kernel's 4-byte loads; D > 64 needs two load
    instructions per row."""
    c, orc, torch, use = env
    use(dim)
    from paper_1407_7737_amd.inputs import population
    n = 333  # 20 full groups of 16 rows and a ragged tail of 13
    for fid in (11, 14, 16, 19):  # direct loads (x3 and x6) and the staged pairwise path
        say(f"[unaligned] dim={dim} fid={fid} n={n}")
        p = orc.basic(fid, dim, SEED)
        x32 = population(n, dim, seed=dim + fid).astype(np.float32)
        buf = torch.zeros(n * dim + 1, dtype=torch.float32, device="cuda")
        xv = buf[1:].view(n, dim)
        xv.copy_(torch.from_numpy(x32))
        assert xv.data_ptr() % 16 != 0
        f = c.func_evaluatef(fid, xv).cpu().numpy()
        x32w = x32.astype(np.float64)
        check32(orc, fid, p, x32w, f, p(x32w), "unaligned")


def test_outputs_beyond_n_untouched_and_zero_rows(env):
    c, orc, torch, use = env
    use(30)
    from paper_1407_7737_amd.inputs import population
    x = torch.from_numpy(population(40, 30, seed=3)).cuda()
    out = torch.full((64,), -7.0, dtype=torch.float64, device="cuda")
    c.func_evaluate(2, x[:33], out=out)
    torch.cuda.synchronize()
    assert torch.all(out[33:] == -7.0)
    c.func_evaluate(2, x[:0], out=out)  # n = 0 is a no-op
    torch.cuda.synchronize()
    assert torch.all(out[33:] == -7.0)


def test_error_codes_on_device(env):
    c, orc, torch, use = env
    use(10, maxc=100)
    x = torch.zeros((101, 10), dtype=torch.float64, device="cuda")
    out = torch.zeros(101, dtype=torch.float64, device="cuda")
    assert c.lib.func_evaluate(0, x.data_ptr(), 101, out.data_ptr()) == c.CUROB_E_CAPACITY
    assert c.lib.func_evaluate(0, None, 5, out.data_ptr()) == c.CUROB_E_ARG
    assert c.lib.func_evaluate(0, x.data_ptr(), -1, out.data_ptr()) == c.CUROB_E_ARG
    assert c.lib.func_evaluate(999, x.data_ptr(), 5, out.data_ptr()) == c.CUROB_E_FID
    assert c.lib.initialize(10, 100, 0) == c.CUROB_E_STATE
    assert c.lib.curob_set_mode(7) == c.CUROB_E_ARG
    assert c.lib.curob_define_basic(5, 11, 1.0, 0.0, 1) == c.CUROB_E_ARG  # id outside the custom range


def test_host_wrappers_match_device_calls(env):
    c, orc, torch, use = env
    use(50, maxc=2000)
    from paper_1407_7737_amd.inputs import population
    x = population(777, 50, seed=5)
    for fid in (2, 9, 19):
        say(f"[host] fid={fid}")
        d = c.func_evaluate(fid, torch.from_numpy(x).cuda()).cpu().numpy()
        h = c.h_func_evaluate(fid, x)
        assert np.array_equal(d, h)
        df = c.func_evaluatef(fid, torch.from_numpy(x.astype(np.float32)).cuda()).cpu().numpy()
        hf = c.h_func_evaluatef(fid, x.astype(np.float32))
        assert np.array_equal(df, hf)


def test_wrong_row_width_is_rejected(env):
    c, orc, torch, use = env
    use(30)
    x = torch.zeros((4, 29), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        c.func_evaluatef(0, x)
    with pytest.raises(ValueError):
        c.get_problem(0, 29)
    assert c.get_dim() == (30, 1 << 18)


def test_context_structure_equals_host_generator(env):
    """curob_get_* on the initialised library describe the problems it evaluates; they equal
    the host-only generator's output (itself checked against the oracle without a GPU)."""
    c, orc, torch, use = env
    use(30)
    for fid, comps in ((11, [-1]), (25, [-1]), (31, [0, 1, 2]), (35, [0, 1, 2])):
        for comp in comps:
            a = c.get_structure(fid, comp)
            b = c.generate_structure(fid, 30, SEED, comp)
            assert a.keys() == b.keys()
            for k in a:
                if k == "blocks":
                    assert all(np.array_equal(u, v) for u, v in zip(a[k], b[k]))
                else:
                    assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), (fid, comp, k)
    for fid in (29, 33, 36):
        assert all(np.array_equal(u, v) for u, v in zip(c.get_composition(fid), c.generate_composition(fid, 30, SEED)))


def test_library_problem_equals_oracle_problem(env):
    c, orc, torch, use = env
    use(64)
    for fid in (0, 11, 14, 16):
        o, R = c.get_problem(fid, 64)
        p = orc.basic(fid, 64, SEED)
        assert np.array_equal(o, p.shift())
        assert np.abs(R - p.rotation()).max() <= 1e-13


def test_custom_basic_rastrigin_at_unit_scale(env):
    """Rastrigin with z = R(x - o) (scale 1), the plain FP64 workload at D = 10, N = 1000."""
    c, orc, torch, use = env
    use(10, maxc=1000)
    from paper_1407_7737_amd.inputs import population
    c.define_basic(64, 11, 1.0, 0.0, True)
    p = orc.custom_basic(64, 11, 10, SEED, 1.0, 0.0, True)
    x = population(1000, 10, seed=0)
    f = c.func_evaluate(64, torch.from_numpy(x).cuda()).cpu().numpy()
    assert rel_err(f, p(x)).max() <= TOL64
    sph = orc.basic(0, 10, SEED)
    f0 = c.func_evaluate(0, torch.from_numpy(x).cuda()).cpu().numpy()
    assert rel_err(f0, sph(x)).max() <= TOL64


def test_nondefault_stream(env):
    c, orc, torch, use = env
    use(100)
    from paper_1407_7737_amd.inputs import population
    x = torch.from_numpy(population(5000, 100, seed=9).astype(np.float32)).cuda()
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        f = c.func_evaluatef(11, x)
    s.synchronize()
    g = c.func_evaluatef(11, x)
    torch.cuda.synchronize()
    assert torch.equal(f, g)


@pytest.mark.parametrize("fid", [0, 2, 9, 10, 11, 14, 16, 19])
def test_full_size_d100_n2p18(env, fid):
    """The measured workload (D = 100, N = 2^18) in the launch configuration the bench uses
    (default split mode), and the plain FP32 mode beside it, every row compared with the
    oracle; the FP64 path on the same points."""
    c, orc, torch, use = env
    use(100)
    from paper_1407_7737_amd.inputs import population
    say(f"[full] fid={fid}")
    n = 1 << 18
    x32 = population(n, 100, seed=0, dtype=np.float32)
    x64 = x32.astype(np.float64)
    p = orc.basic(fid, 100, SEED)
    ref = p(x64, threads=16)
    dx32 = torch.from_numpy(x32).cuda()
    fs = c.func_evaluatef(fid, dx32).cpu().numpy()
    c.set_mode(c.MODE_FP32)
    fp = c.func_evaluatef(fid, dx32).cpu().numpy()
    c.set_mode(c.MODE_SPLIT)
    f64 = c.func_evaluate(fid, torch.from_numpy(x64).cuda()).cpu().numpy()
    e64 = rel_err(f64, ref)
    es = check32(orc, fid, p, x64, fs, ref, "split-full")
    ep = check32(orc, fid, p, x64, fp, ref, "fp32-full")
    say(f"[full] fid={fid} split max {es:.3e}; fp32 max {ep:.3e}; fp64 max {e64.max():.3e}")
    assert e64.max() <= TOL64
