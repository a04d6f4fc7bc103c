"""Small populations in the latency regime (N = 50, D in {10, 32, 64, 96}: the paper's own
setting of many small evaluation calls), evaluated inside a captured HIP graph.

The library's evaluation calls enqueue kernels only (no allocation, copy or memset), so torch's
stream capture records them.  Each graph is replayed several times with eager work and
synchronisations in between; every replay must equal the eager result bit for bit, and the
eager result must meet the oracle bar.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SEED = 0
TOL32 = 1e-4
TOL64 = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def schwefel_edge_rows(orc, p, x):
    s, c, _ = orc.table_xform(16)
    y = s * (x - p.shift()[None, :])
    w = np.abs(y @ p.rotation().T + c + 420.9687462275036)
    d = np.where(w >= 750.0, np.abs(w - 500.0 * np.round(w / 500.0)), np.inf)
    delta = 64.0 * 2.0 ** -24 * (1.0 + np.linalg.norm(y, axis=1, keepdims=True))
    return (d < delta).any(axis=1)


@pytest.mark.parametrize("dim", [10, 32, 64, 96])
def test_graph_replay_matches_eager(dim):
    import torch
    assert torch.cuda.is_available()
    import oracle
    import paper_1407_7737_amd as c
    from paper_1407_7737_amd.inputs import population
    c.initialize(dim, 64, SEED)
    try:
        fids = [0, 2, 9, 11, 14, 16, 19]
        x64 = population(50, dim, seed=dim)
        x32 = x64.astype(np.float32)
        dx32 = torch.from_numpy(x32).cuda()
        dx64 = torch.from_numpy(x64).cuda()
        o32 = {f: torch.empty(50, device="cuda") for f in fids}
        o64 = {f: torch.empty(50, device="cuda", dtype=torch.float64) for f in fids}
        # eager results
        e32 = {f: c.func_evaluatef(f, dx32).clone() for f in fids}
        e64 = {f: c.func_evaluate(f, dx64).clone() for f in fids}
        torch.cuda.synchronize()
        for f in fids:
            p = oracle.basic(f, dim, SEED)
            ref = p(x64)
            assert np.max(np.abs(e64[f].cpu().numpy() - ref) / np.maximum(1, np.abs(ref))) <= TOL64
            x32w = x32.astype(np.float64)
            ref32 = p(x32w)
            err = np.abs(e32[f].cpu().numpy() - ref32) / np.maximum(1, np.abs(ref32))
            if f == 16:
                # rotated Schwefel: only rows with a component of w = z + 420.97 within FP32
                # rounding (64 ulp of |y|) of a g1 jump at |w| = 1000, 1500, ... are exempt
                err = np.where(schwefel_edge_rows(oracle, p, x32w), 0.0, err)
            assert err.max() <= TOL32, (dim, f, float(err.max()))
        # one graph with every call
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                for f in fids:
                    c.func_evaluatef(f, dx32, out=o32[f])
                    c.func_evaluate(f, dx64, out=o64[f])
        torch.cuda.current_stream().wait_stream(s)
        for r in range(3):
            for f in fids:
                o32[f].fill_(np.nan)
                o64[f].fill_(np.nan)
            _ = torch.ones(1000, device="cuda").cumsum(0)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            for f in fids:
                assert torch.equal(o32[f], e32[f]), (dim, f, r)
                assert torch.equal(o64[f], e64[f]), (dim, f, r)
        say(f"[graph] dim={dim}: {len(fids)} formulas x 2 paths, 3 replays equal the eager results")
        del g
    finally:
        torch.cuda.synchronize()
        c.set_stream(None)
        c.dispose()
