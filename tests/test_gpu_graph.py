"""The step replayed as a HIP graph (sgs_options.graph) against the same
steps enqueued kernel by kernel: the same kernels in the same order, so the
energies and states must agree bit for bit, on every replay, with eager work
of the program (table evaluations, torch operations, synchronizations)
between replays, and after a change of dtau (a new capture)."""

import sys

import numpy as np
import pytest

import sgs_inputs as si

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pair(hams, gams, **kw):
    from paper_2105_01088_amd import SGS, default_options
    eager = SGS(hams, gams, options=default_options(**kw))
    graph = SGS(hams, gams, options=default_options(graph=1, **kw))
    return eager, graph


def _same(a, b):
    for p in range(a.nprob):
        assert torch.equal(a.gammas(p), b.gammas(p))


@pytest.mark.parametrize("weight,update", [(0, 0), (1, 0), (1, 1)])
def test_graph_replays_match_eager_single(weight, update):
    ham, gam, cfg = si.config_problem("anderson_L7_R4")
    _say(f"[graph] anderson L=7 R=4 weight={weight} update={update}")
    eager, graph = _pair([ham], [gam], weight=weight, update=update)
    for rnd, (dtau, k) in enumerate([(0.05, 5), (0.05, 3), (0.03, 4), (0.05, 2)]):
        ee = eager.step(dtau, k)
        eg = graph.step(dtau, k)
        torch.cuda.synchronize()
        assert torch.equal(ee, eg), f"round {rnd}"
        _same(eager, graph)
        # eager work between replays: tables of the graph context, torch ops
        la, ar, ep = graph.pair_eval()
        la2, ar2, ep2 = eager.pair_eval()
        assert torch.equal(la, la2) and torch.equal(ep, ep2)
        x = torch.randn(257, 257, dtype=torch.float64, device="cuda:0")
        (x @ x).sum().item()
    assert eager.status() == 0 and graph.status() == 0
    eager.close()
    graph.close()


def test_graph_replays_match_eager_batch():
    """Three problems of different sizes on the worker streams: one graph
    launch per step for the whole batch."""
    hams, gams = [], []
    for L, R, seed in [(5, 3, 1), (20, 5, 2), (11, 4, 3)]:
        h = si.anderson(L, 1.2, 0.5)
        hams.append(h)
        gams.append(si.random_states(h.N, R, seed))
    _say("[graph] batch of 3 problems")
    eager, graph = _pair(hams, gams, weight=1)
    for k in (4, 1, 3):
        ee = eager.step(0.05, k)
        eg = graph.step(0.05, k)
        torch.cuda.synchronize()
        assert torch.equal(ee, eg)
        _same(eager, graph)
        E1, _ = eager.energy()
        E2, _ = graph.energy()
        assert torch.equal(E1, E2)
    assert eager.status() == 0 and graph.status() == 0
    eager.close()
    graph.close()


def test_graph_more_steps_than_the_energy_ring():
    """More replays in one call than the 1024-entry energy ring: the energies
    are copied out in chunks."""
    ham = si.anderson(1, 1.0, 0.5)
    gam = si.random_states(ham.N, 2, seed=2)
    _say("[graph] 1100 steps")
    eager, graph = _pair([ham], [gam], weight=1)
    ee = eager.step(0.01, 1100)
    eg = graph.step(0.01, 1100)
    torch.cuda.synchronize()
    assert torch.equal(ee, eg)
    _same(eager, graph)
    eager.close()
    graph.close()
