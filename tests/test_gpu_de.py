"""The optimiser in the loop (curob_de_run): DE/rand/1/bin on the GPU in the paper's small-batch
setting (50 candidates per evaluation call, D in {10, 32, 64, 96}, Sec. 2).

- FP64 populations: the GPU run equals the oracle's DE (same specification, FP64 formulas) bit
  for bit in the vectors and to 1e-10 in the values, provided no selection decision of the
  oracle run was closer than 1e-9 (relative) -- the FP64 path's error could flip such a one.
- K generations captured in one graph: each replay equals the same generations run eagerly,
  bit for bit, on both paths, and replays continue the generation sequence.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NP = 50
SEED = 0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    import oracle
    import paper_1407_7737_amd as c
    yield c, oracle, torch


@pytest.mark.parametrize("dim", [10, 32, 64, 96])
def test_de_fp64_matches_oracle(env, dim):
    c, orc, torch = env
    from paper_1407_7737_amd.inputs import population
    c.initialize(dim, 64, SEED)
    try:
        for fid in (11, 19):
            say(f"[de] dim={dim} fid={fid} fp64 vs oracle")
            pop0 = population(NP, dim, seed=100 + dim)
            de = c.DE(fid, torch.from_numpy(pop0).cuda(), F=0.5, CR=0.9, seed=77, fp64=True)
            de.run(30)
            torch.cuda.synchronize()
            p = orc.basic(fid, dim, SEED)
            pop, fit = pop0.copy(), p(pop0)
            margin = p.de_run(pop, fit, 0.5, 0.9, 77, 0, 30)
            assert margin > 1e-9, (dim, fid, margin)  # no decision within the FP64 path's error
            assert np.array_equal(de.pop.cpu().numpy(), pop), (dim, fid)
            got = de.fit.cpu().numpy()
            assert np.max(np.abs(got - fit) / np.maximum(1.0, np.abs(fit))) <= 1e-10
            assert int(de.gen.item()) == 30
            say(f"[de] dim={dim} fid={fid}: best {fit.min():.6g} after 30 generations (from {p(pop0).min():.6g})")
    finally:
        torch.cuda.synchronize()
        c.set_stream(None)
        c.dispose()


@pytest.mark.parametrize("dim", [10, 96])
@pytest.mark.parametrize("fp64", [False, True])
def test_de_graph_replay_equals_eager(env, dim, fp64):
    c, orc, torch = env
    from paper_1407_7737_amd.inputs import population
    c.initialize(dim, 64, SEED)
    try:
        dt = np.float64 if fp64 else np.float32
        pop0 = torch.from_numpy(population(NP, dim, seed=5).astype(dt)).cuda()
        eager = c.DE(11, pop0, seed=3, fp64=fp64)
        graph = c.DE(11, pop0, seed=3, fp64=fp64)
        graph.capture(10)
        for rep in range(3):
            eager.run(10)
            _ = torch.ones(4096, device="cuda").cumsum(0)  # unrelated eager work between replays
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            say(f"[de-graph] dim={dim} fp64={fp64} replay {rep}: gen {int(graph.gen.item())}")
            assert torch.equal(graph.pop, eager.pop) and torch.equal(graph.fit, eager.fit), (dim, fp64, rep)
            assert int(graph.gen.item()) == int(eager.gen.item()) == 10 * (rep + 1)
        # the stored values are the values of the stored vectors
        f = (c.func_evaluate if fp64 else c.func_evaluatef)(11, eager.pop)
        torch.cuda.synchronize()
        assert torch.equal(f, eager.fit)
        del graph.graph
    finally:
        torch.cuda.synchronize()
        c.set_stream(None)
        c.dispose()


def test_de_argument_checks(env):
    c, orc, torch = env
    c.initialize(10, 64, SEED)
    try:
        x = torch.zeros((NP, 10), dtype=torch.float64, device="cuda")
        g = torch.zeros(1, dtype=torch.int64, device="cuda")
        p = x.data_ptr()
        assert c.lib.curob_de_run(11, 1, 3, 0.5, 0.9, 0, p, p, p, p, g.data_ptr(), 1) == c.CUROB_E_ARG
        assert c.lib.curob_de_run(11, 1, NP, 0.0, 0.9, 0, p, p, p, p, g.data_ptr(), 1) == c.CUROB_E_ARG
        assert c.lib.curob_de_run(11, 1, NP, 0.5, 1.5, 0, p, p, p, p, g.data_ptr(), 1) == c.CUROB_E_ARG
        assert c.lib.curob_de_run(11, 1, 65, 0.5, 0.9, 0, p, p, p, p, g.data_ptr(), 1) == c.CUROB_E_CAPACITY
        assert c.lib.curob_de_run(11, 1, NP, 0.5, 0.9, 0, p, p, p, p, None, 1) == c.CUROB_E_ARG
    finally:
        c.dispose()
