"""func_evaluatef_noalloc (the allocation-free FP32 entry point) against func_evaluatef.

Both run the same kernels; the allocation-free call takes its scratch from the library's static
device array and evaluates in passes of as many rows as fit there, so its results must equal the
allocating call's bit for bit.  Two calls in a row, the second on fewer rows, per problem and
mode.  At D = 1000 (a basic function with pair terms, one without, a paper hybrid and a paper
composition): the FP32-MFMA mode runs the tiled kernels, whose partial sums, pairwise z and
packed operands live in the scratch; the default split mode runs the row-resident kernels,
which need none.  At D = 100: resident-kernel functions (no scratch) and a paper composition,
whose component values pass through the scratch before the blend.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(c, torch, fid, x, out_len):
    """Both entry points on x; the outputs are pre-filled so untouched entries are visible."""
    n = x.shape[0]
    ref = torch.full((out_len,), -1.0, device="cuda")
    got = torch.full((out_len,), -2.0, device="cuda")
    c.set_stream(torch.cuda.current_stream())
    c.check(c.lib.func_evaluatef(int(fid), x.data_ptr(), n, ref.data_ptr()))
    c.check(c.lib.func_evaluatef_noalloc(int(fid), x.data_ptr(), n, got.data_ptr()))
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


@pytest.mark.parametrize("dim,fids,modes", [(1000, [14, 19, 25, 32], ("MODE_FP32", "MODE_SPLIT")),
                                            (100, [11, 16, 32], ("MODE_SPLIT",))])
def test_noalloc_matches_allocating_call(dim, fids, modes):
    import torch
    assert torch.cuda.is_available()
    import oracle
    import paper_1407_7737_amd as c
    from paper_1407_7737_amd.inputs import population
    c.initialize(dim, 12000, 0)
    try:
        big = torch.from_numpy(population(9000, dim, seed=1, dtype=np.float32)).cuda()
        small = torch.from_numpy(population(1234, dim, seed=2, dtype=np.float32)).cuda()
        for mode in modes:
            c.set_mode(getattr(c, mode))
            for fid in fids:
                for tag, x in (("first", big), ("second, smaller", small)):
                    say(f"[noalloc] dim={dim} {mode} fid={fid} {tag} call n={x.shape[0]}")
                    ref, got = _run(c, torch, fid, x, 9000)
                    n = x.shape[0]
                    assert np.array_equal(got[:n], ref[:n]), (dim, mode, fid, n,
                                                              float(np.abs(got[:n] - ref[:n]).max()))
                    assert np.all(got[n:] == -2.0)
                # and the FP32 bar against the oracle on a few rows of the last call
                p = oracle.fid_problem(fid, dim, 0)
                xw = small[:16].cpu().numpy().astype(np.float64)
                want = p(xw, threads=16)
                err = np.abs(got[:16] - want) / np.maximum(1.0, np.abs(want))
                assert err.max() <= 1e-4 or fid == 16, (mode, fid, float(err.max()))
        c.set_mode(c.MODE_SPLIT)
        # a problem that needs no scratch at all through the same entry point, n = 0 included
        assert c.lib.func_evaluatef_noalloc(11, None, 0, None) == c.CUROB_OK
        assert c.lib.func_evaluatef_noalloc(999, big.data_ptr(), 5, big.data_ptr()) == c.CUROB_E_FID
    finally:
        torch.cuda.synchronize()
        c.set_stream(None)
        c.dispose()
