"""Several independent problems in one context (the batched workload): every
problem's step, tables and observables must equal the oracle's for that
problem alone, with the problems run on one stream or concurrently on
several (sharing scratch regions between problems of one stream)."""

import sys

import numpy as np
import pytest

import sgs_inputs as si
from oracle import observables as ob
from oracle import sgs as osgs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_TAB = 1e-9
TOL_GAMMA = 1e-10
TOL_E = 1e-10


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _problems():
    out = []
    for L, R, seed, U, V in [(3, 4, 1, 1.3, 0.6), (8, 3, 2, 1.0, 0.5), (5, 5, 3, 2.0, 0.4),
                             (12, 2, 4, 0.7, 0.3), (2, 1, 5, 1.0, 0.5)]:
        ham = si.anderson(L, U, V)
        out.append((ham, si.random_states(ham.N, R, seed)))
    ham = si.two_channel_kondo(2, 0.5)
    out.append((ham, si.random_states(ham.N, 3, 6)))
    return out


def _ctx(probs, **kw):
    from paper_2105_01088_amd import SGS, default_options
    return SGS([h for h, _ in probs], [g for _, g in probs], options=default_options(**kw))


@pytest.mark.parametrize("streams", [1, 4, 8])
def test_batched_steps_match_oracle(streams):
    probs = _problems()
    _say(f"[batched] {len(probs)} problems, streams={streams}, 2 steps")
    ctx = _ctx(probs, weight=1, streams=streams)
    e = ctx.step(0.05, 2).cpu().numpy().reshape(2, len(probs))
    assert ctx.status() == 0
    for p, (ham, gam) in enumerate(probs):
        g = gam
        for k in range(2):
            r = osgs.step(ham, g, 0.05, mode="unit")
            assert abs(e[k, p] - r.E) < TOL_E * abs(r.E)
            g = r.gammas
        assert np.abs(ctx.gammas(p).cpu().numpy() - g).max() < TOL_GAMMA
    ctx.close()


def test_batched_tables_energy_and_observables():
    probs = _problems()
    _say("[batched] tables, energies, observables")
    ctx = _ctx(probs, streams=4)
    la, ar, ep = ctx.pair_eval()
    assert ctx.status() == 0
    la, ar = la.cpu().numpy(), ar.cpu().numpy()
    ep = ep.cpu().numpy()
    E, lam = ctx.energy()
    E = E.cpu().numpy()
    off = 0
    for p, (ham, gam) in enumerate(probs):
        R = gam.shape[0]
        ref = osgs.pair_tables(ham, gam)
        tl = la[off:off + R * R].reshape(R, R)
        te = (ep[2 * off:2 * (off + R * R):2] + 1j * ep[2 * off + 1:2 * (off + R * R):2]).reshape(R, R)
        offd = ~np.eye(R, dtype=bool)
        if R > 1:
            assert np.abs(tl - ref.logabs)[offd].max() < TOL_TAB * max(1.0, np.abs(ref.logabs).max())
        assert np.abs(te - ref.eps).max() < TOL_TAB * max(1.0, np.abs(ref.eps).max())
        Eref, _, _ = osgs.energy(ham, gam)
        assert abs(E[p] - Eref) < TOL_E * abs(Eref)
        off += R * R
    # observables of problems that share a stream: tables are re-evaluated per problem
    for p in (2, 0, 5, 1):
        ham, gam = probs[p]
        L_sites = ham.N // 2 - 1
        polys = [si.spin_dot_poly((0, 1), (2 * r, 2 * r + 1)) for r in range(0, min(3, L_sites) + 1)]
        got = ctx.expectations(polys, problem=p)
        Eref, lamr, tab = osgs.energy(ham, gam)
        ref = np.array([ob.expectation(gam, lamr, tab.G, q) for q in polys])
        assert np.abs(got - ref).max() < 1e-9 * max(1.0, np.abs(ref).max())
        s2 = ctx.renyi2(4, problem=p)
        assert abs(s2 - ob.renyi2(gam, lamr, tab.G, 4)) < 1e-9
    ctx.close()


def test_batched_workload_sample_one_step():
    """A batch of 8 from the batched-workload generator (uneven n and R, L
    limited to 20..60 so the oracle stays quick), one step each."""
    probs = [(h, g) for h, g, _ in si.batched_problems(0, count=8, L_range=(20, 60))]
    _say("[batched] 8 generated problems, one step")
    ctx = _ctx(probs, weight=1)
    e = ctx.step(0.05, 1).cpu().numpy()
    assert ctx.status() == 0
    for p, (ham, gam) in enumerate(probs):
        r = osgs.step(ham, gam, 0.05, mode="unit")
        assert abs(e[p] - r.E) < TOL_E * abs(r.E)
        assert np.abs(ctx.gammas(p).cpu().numpy() - r.gammas).max() < TOL_GAMMA
    ctx.close()
