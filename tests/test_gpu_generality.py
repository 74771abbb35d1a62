"""Hamiltonians beyond the benchmark chains, through the C ABI against the
oracle: the Anderson bath with the Wilson tail of the Fig. 4 caption
(20 sites, t_n = 1.2^-n), and a dense random skew A with quartic words
(every entry of A nonzero: the sparse traces, the Fock products and the
elementwise force terms see full columns).  Tolerances as the other parity
tests: 1e-10 on Gamma and E for a step, 1e-9 on the variance."""

import sys

import numpy as np
import pytest

import sgs_inputs as si
from oracle import observables as ob
from oracle import sgs as osgs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_GAMMA = 1e-10
TOL_E = 1e-10


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dense_ham(N, seed, nq=2):
    rng = np.random.default_rng(seed)
    n = 2 * N
    z = rng.standard_normal((n, n)) / np.sqrt(n)
    A = 0.5 * (z - z.T)
    words = np.array([np.sort(rng.choice(n, size=4, replace=False)) for _ in range(nq)], dtype=np.int32)
    vals = rng.uniform(0.2, 0.8, size=nq)
    return si.MajoranaHamiltonian(N=N, A=A, quartic_idx=words, quartic_val=vals, e0=0.3)


def _step_case(ham, gam, weight, nsteps):
    from paper_2105_01088_amd import SGS, default_options
    ctx = SGS([ham], [gam], options=default_options(weight=weight))
    e = ctx.step(0.05, nsteps).cpu().numpy()
    assert ctx.status() == 0
    g = gam
    es = []
    for _ in range(nsteps):
        r = osgs.step(ham, g, 0.05, mode="printed" if weight == 0 else "unit")
        es.append(r.E)
        g = r.gammas
    assert np.abs(e - es).max() < TOL_E * np.abs(es).max()
    assert np.abs(ctx.gammas(0).cpu().numpy() - g).max() < TOL_GAMMA
    v = ctx.variance()
    assert ctx.status() == 0
    E, lam, tab = osgs.energy(ham, g)
    ref = ob.hamiltonian_variance_trace(ham, g, lam, tab.G)
    assert abs(v[1] - ref[1]) < 1e-9 * max(1.0, abs(ref[1]))
    assert abs(v[2] - ref[2]) < 3e-9 * max(1.0, abs(ref[1]))
    ctx.close()


def test_wilson_tail_steps():
    ham = si.anderson(10, 1.0, 0.45, wilson_tail=si.wilson_hoppings(20, 1.2))
    gam = si.random_states(ham.N, 4, 5)
    _say(f"[general] Wilson tail n={ham.n} R=4")
    _step_case(ham, gam, 1, 3)


@pytest.mark.parametrize("weight", [0, 1])
def test_dense_hamiltonian_steps(weight):
    ham = _dense_ham(12, 3)
    gam = si.random_states(ham.N, 3, 8)
    _say(f"[general] dense A n={ham.n} R=3 weight={weight}")
    _step_case(ham, gam, weight, 2)
