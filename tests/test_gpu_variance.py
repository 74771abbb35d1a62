"""Variance of the Hamiltonian, Eq. (residual): delta_H^2 = <H^2> - <H>^2,
through the C ABI (SGS_OBS_VARIANCE) against the oracle.

Small systems against the word expansion of H^2 (``hamiltonian_variance``):
Anderson n = 16 with R = 1 and 3, the two-channel Kondo model (several
quartic words: 6- and 8-Majorana Pfaffians) with R = 3, a ragged n = 132
over several tiles, the exact Gaussian ground state of a quadratic H
(delta_H^2 = 0), and a dense A with odd R.  R = 32 (the largest) and full
size (n = 400, R = 16) against the matrix form (``hamiltonian_variance_trace``,
itself pinned to the word expansion), the latter before and after 5 steps.

Tolerance: <H> and <H^2> are sums of lambda_mu^* lambda_b G_mb <.>_t, so
they inherit the tables' relative accuracy (1e-9, as the other
observables); delta_H^2 is their difference: 3e-9 <H^2> absolute.
"""

import sys

import numpy as np
import pytest

import sgs_inputs as si
from oracle import observables as ob
from oracle import sgs as osgs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-9


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _ctx(ham, gam):
    from paper_2105_01088_amd import SGS, default_options
    return SGS([ham], [gam], options=default_options(weight=1))


def _check(got, ref):
    e1, e2, var = got
    r1, r2, rv = ref
    assert abs(e1 - r1) < TOL * max(1.0, abs(r1))
    assert abs(e2 - r2) < TOL * max(1.0, abs(r2))
    assert abs(var - rv) < 3 * TOL * max(1.0, abs(r2))


CASES = [("anderson", 3, 1, 4), ("anderson", 3, 3, 2), ("tck", 1, 3, 7), ("anderson", 32, 2, 1)]


@pytest.mark.parametrize("model,L,R,seed", CASES)
def test_variance_matches_oracle(model, L, R, seed):
    ham = si.anderson(L, 1.3, 0.7) if model == "anderson" else si.two_channel_kondo(L, 0.9, U=2.0)
    gam = si.random_states(ham.N, R, seed)
    _say(f"[variance] {model} L={L} n={ham.n} R={R}")
    ctx = _ctx(ham, gam)
    got = ctx.variance()
    assert ctx.status() == 0
    E, lam, tab = osgs.energy(ham, gam)
    ref = ob.hamiltonian_variance(ham, gam, lam, tab.G) if ham.n <= 32 else \
        ob.hamiltonian_variance_trace(ham, gam, lam, tab.G)
    _check(got, ref)
    Eg, _ = ctx.energy()
    assert abs(got[0] - Eg.cpu().item()) < TOL * max(1.0, abs(got[0]))
    ctx.close()


def test_variance_largest_R():
    """R = 32 (the most the variance takes): 528 blocks b <= mu, the others
    taken as their conjugates."""
    ham = si.anderson(3, 1.3, 0.7)
    gam = si.random_states(ham.N, 32, 11)
    _say(f"[variance] anderson n={ham.n} R=32")
    ctx = _ctx(ham, gam)
    got = ctx.variance()
    assert ctx.status() == 0
    E, lam, tab = osgs.energy(ham, gam)
    _check(got, ob.hamiltonian_variance_trace(ham, gam, lam, tab.G))
    ctx.close()


def test_variance_dense_A():
    """Every column of A full (the longest column walks), two quartic words,
    odd R; against the word expansion."""
    rng = np.random.default_rng(3)
    N = 12
    n = 2 * N
    z = rng.standard_normal((n, n)) / np.sqrt(n)
    words = np.array([np.sort(rng.choice(n, size=4, replace=False)) for _ in range(2)], dtype=np.int32)
    ham = si.MajoranaHamiltonian(N=N, A=0.5 * (z - z.T), quartic_idx=words,
                                 quartic_val=rng.uniform(0.2, 0.8, size=2), e0=0.3)
    gam = si.random_states(ham.N, 5, 2)
    _say(f"[variance] dense A n={ham.n} R=5")
    ctx = _ctx(ham, gam)
    got = ctx.variance()
    assert ctx.status() == 0
    E, lam, tab = osgs.energy(ham, gam)
    _check(got, ob.hamiltonian_variance(ham, gam, lam, tab.G))
    ctx.close()


def test_variance_zero_on_gaussian_eigenstate():
    ham = si.anderson(7, 0.0, 0.7)
    w, v = np.linalg.eigh(1j * ham.A)
    gam = (-1j * (v * np.sign(w)) @ v.conj().T).real
    gam = 0.5 * (gam - gam.T)[None]
    _say(f"[variance] eigenstate n={ham.n}")
    ctx = _ctx(ham, gam)
    e1, e2, var = ctx.variance()
    assert ctx.status() == 0
    assert abs(var) < 3 * TOL * e2
    assert abs(e1 - (ham.e0 - np.abs(w).sum())) < TOL * max(1.0, abs(e1))
    ctx.close()


def test_variance_full_size():
    """n = 400, R = 16: the seeded states, then after 5 steps."""
    ham, gam, cfg = si.config_problem("anderson_L99_R16")
    _say("[variance] anderson_L99_R16 (n=400, R=16)")
    ctx = _ctx(ham, gam)
    got = ctx.variance()
    assert ctx.status() == 0
    E, lam, tab = osgs.energy(ham, gam)
    _check(got, ob.hamiltonian_variance_trace(ham, gam, lam, tab.G))
    ctx.step(0.05, 5)
    got2 = ctx.variance()
    assert ctx.status() == 0
    g5 = ctx.gammas(0).cpu().numpy()
    E5, lam5, tab5 = osgs.energy(ham, g5)
    _check(got2, ob.hamiltonian_variance_trace(ham, g5, lam5, tab5.G))
    ctx.close()
