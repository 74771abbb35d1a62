"""Renyi-2 entropy (Eq. S2_SGS, App. B) on the GPU, through the C ABI, against
the oracle's definition (all R^4 terms, each a Pfaffian of order 2 nA): the
batched block form of Eq. (pfMA), the split form of Eq. (TrArho2_final) and
the automatic choice between them, for subsystems beyond the on-chip path
(nA > 32), and for states whose Gamma restricted to A is singular (Majorana
pairs across the cut), where only the block form applies.

Tolerance 1e-9 relative to max(1, |S_2|): the tables enter through lambda and
G (pinned at 1e-9 by the pair-table tests); the split form adds the rounding
of one block inverse, bounded by its condition number (at most 1e6 in the
automatic choice) times the unit roundoff."""

import sys

import numpy as np
import pytest

import sgs_inputs as si
from oracle import observables as ob
from oracle import sgs as osgs
from oracle.pfaffian import pfaffian_log

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-9


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _ctx(ham, gam, **kw):
    from paper_2105_01088_amd import SGS, default_options
    return SGS([ham], [gam], options=default_options(**kw))


def _check(ham, gam, nA, method, **kw):
    ctx = _ctx(ham, gam, **kw)
    got = ctx.renyi2(nA, method=method)
    st = ctx.status()
    ctx.close()
    E, lam, tab = osgs.energy(ham, gam)
    ref = ob.renyi2(gam, lam, tab.G, nA)
    assert st == 0
    assert abs(got - ref) < TOL * max(1.0, abs(ref)), (got, ref)
    return got


def _crossing_state(n):
    """Pure, even state with Majorana pairs (1, 2), (3, 4), ..., (n-1, 0): for
    any even cut nA, Majoranas 0 and nA-1 are paired across it, so Gamma on A
    has two zero rows."""
    g = np.zeros((n, n))
    for j in range(1, n - 1, 2):
        g[j, j + 1], g[j + 1, j] = 1.0, -1.0
    g[0, n - 1], g[n - 1, 0] = 1.0, -1.0  # the cyclic relabelling is odd: this sign keeps Pf = +1
    la, ph = pfaffian_log(g)
    assert abs(la) < 1e-12 and abs(ph - 1.0) < 1e-12
    return g


@pytest.mark.parametrize("method", [1, 2])
@pytest.mark.parametrize("nA", [4, 16])
def test_batched_methods_small_subsystem(nA, method):
    """The batched block and split forms where the on-chip path also applies."""
    ham = si.anderson(3, 1.3, 0.6)
    gam = si.random_states(ham.N, 4, 3)
    _say(f"[renyi] n={ham.n} R=4 nA={nA} method={method}")
    _check(ham, gam, nA, method)


@pytest.mark.parametrize("nA", [32, 34, 48, 64, 98])
def test_large_subsystems(nA):
    """Impurity plus j sites (nA = 4 (j + 1)) and beyond, n = 100, R = 3."""
    ham = si.anderson(24, 1.0, 0.5)
    gam = si.random_states(ham.N, 3, 11)
    _say(f"[renyi] n={ham.n} R=3 nA={nA} auto")
    _check(ham, gam, nA, 0)


@pytest.mark.parametrize("method", [0, 1, 2])
def test_all_methods_agree_at_nA_48(method):
    ham = si.anderson(24, 1.0, 0.5)
    gam = si.random_states(ham.N, 4, 12)
    _say(f"[renyi] n={ham.n} R=4 nA=48 method={method}")
    _check(ham, gam, 48, method)


def test_whole_system_is_pure():
    """Tr rho^2 = 1 for A = the whole system (n = 100), through the batched path."""
    ham = si.anderson(24, 1.0, 0.5)
    gam = si.random_states(ham.N, 3, 13)
    _say(f"[renyi] n={ham.n} whole system")
    ctx = _ctx(ham, gam)
    for method in (0, 1, 2):
        assert abs(ctx.renyi2(ham.n, method=method)) < 1e-10
    ctx.close()


@pytest.mark.parametrize("method", [0, 1, 2])
@pytest.mark.parametrize("nA", [16, 48])
def test_singular_blocks(nA, method):
    """A state with Majorana pairs across the cut: K_aa = Gamma_a on A is
    singular, so terms pairing it with itself need the block form."""
    ham = si.anderson(24, 1.0, 0.5)
    gam = si.random_states(ham.N, 3, 14)
    gam[0] = _crossing_state(ham.n)
    _say(f"[renyi] n={ham.n} crossing state nA={nA} method={method}")
    _check(ham, gam, nA, method)


def test_benchmark_workload_impurity_plus_eight_sites():
    """n = 400, R = 16 (about 16.6k representative terms): S_2 of the
    impurity plus 8 sites (nA = 36) against all 65536 oracle terms."""
    ham, gam, cfg = si.config_problem("anderson_L99_R16")
    _say("[renyi] anderson_L99_R16 nA=36")
    _check(ham, gam, 36, 0, weight=1)


@pytest.mark.parametrize("method", [0, 1, 2])
def test_near_copy_states_nA_48(method):
    """Rotated near-copy states (overlaps of order one): every cross term of
    the rank-4 tensor weighs as much as the diagonal ones, through the
    batched block and split forms at nA = 48."""
    ham = si.anderson(24, 1.0, 0.5)
    gam = si.near_copy_states(ham.N, 3, 1.5, seed=15)
    _say(f"[renyi] near-copy n={ham.n} R=3 nA=48 method={method}")
    _check(ham, gam, 48, method)
