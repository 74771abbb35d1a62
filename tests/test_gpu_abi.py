"""Error codes and optional outputs of the C ABI that need a device: input
validation in sgs_init (skew, pure, even parity, NaN), the device status
word after a singular pair, and the transition matrices of sgs_pair_eval
against the oracle's Delta (Eq. def-delta-matrix)."""

import sys

import numpy as np
import pytest

import sgs_inputs as si
from oracle import gaussian as ga

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SGS_ENOTSKEW, SGS_ENOTPURE, SGS_EPARITY, SGS_ESINGULAR = -2, -3, -4, -5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _init_code(ham, gam):
    from paper_2105_01088_amd import SGS, SGSError, default_options
    try:
        ctx = SGS([ham], [gam], options=default_options())
    except SGSError as e:
        return e.code
    ctx.close()
    return 0


def test_init_accepts_valid_states():
    ham = si.anderson(5, 1.0, 0.5)
    _say("[abi] valid states")
    assert _init_code(ham, si.random_states(ham.N, 3, seed=1)) == 0


def test_init_rejects_non_skew():
    ham = si.anderson(5, 1.0, 0.5)
    gam = si.random_states(ham.N, 3, seed=1)
    gam[1, 2, 5] += 1e-6  # Gamma + Gamma^T = 1e-6 at one entry
    _say("[abi] ENOTSKEW")
    assert _init_code(ham, gam) == SGS_ENOTSKEW


def test_init_rejects_non_pure():
    ham = si.anderson(5, 1.0, 0.5)
    gam = si.random_states(ham.N, 3, seed=1)
    gam[2] *= 0.999  # skew, Gamma^2 = -0.998
    _say("[abi] ENOTPURE")
    assert _init_code(ham, gam) == SGS_ENOTPURE


@pytest.mark.parametrize("state", [0, 2])
def test_init_rejects_odd_parity(state):
    """Exchanging two Majoranas (det = -1) flips Pf Gamma to -1: a pure,
    skew, odd state."""
    ham = si.anderson(5, 1.0, 0.5)
    gam = si.random_states(ham.N, 3, seed=1)
    p = np.arange(ham.n)
    p[[0, 1]] = p[[1, 0]]
    gam[state] = gam[state][np.ix_(p, p)]
    _say(f"[abi] EPARITY (state {state})")
    assert _init_code(ham, gam) == SGS_EPARITY


@pytest.mark.parametrize("where", ["off", "diag"])
def test_init_rejects_nan(where):
    ham = si.anderson(5, 1.0, 0.5)
    gam = si.random_states(ham.N, 3, seed=1)
    if where == "off":
        gam[1, 3, 4] = np.nan
    else:
        gam[0, 2, 2] = np.nan
    _say(f"[abi] NaN ({where})")
    assert _init_code(ham, gam) in (SGS_ENOTSKEW, SGS_ENOTPURE)


def test_singular_pair_sets_status():
    """Gamma_1 = -Gamma_0 (even parity for even N): Gamma_0 + Gamma_1 = 0, so
    the pair's inverse fails and the status word reports it."""
    from paper_2105_01088_amd import SGS, default_options
    ham = si.anderson(3, 1.0, 0.5)  # N = 8
    g0 = si.random_states(ham.N, 1, seed=4)[0]
    gam = np.stack([g0, -g0])
    _say("[abi] ESINGULAR through the status word")
    ctx = SGS([ham], [gam], options=default_options())
    ctx.pair_eval()
    assert ctx.status() == SGS_ESINGULAR
    assert ctx.status() == 0  # reading the status clears it
    ctx.close()


@pytest.mark.parametrize("L,R", [(3, 4), (20, 3)])
def test_pair_eval_delta_output(L, R):
    """Delta^{ba} of every pair a < b, in pair order, against the oracle."""
    from paper_2105_01088_amd import SGS, default_options
    ham = si.anderson(L, 1.1, 0.6)
    gam = si.random_states(ham.N, R, seed=6)
    _say(f"[abi] Delta output n={ham.n} R={R}")
    ctx = SGS([ham], [gam], options=default_options())
    la, ar, ep, dl = ctx.pair_eval(delta=True)
    assert ctx.status() == 0
    d = dl[0].cpu().numpy()
    k = 0
    for a in range(R):
        for b in range(a + 1, R):
            ref = ga.delta(gam[b], gam[a])  # Delta^{ba}
            assert np.abs(d[k] - ref).max() < 1e-10 * max(1.0, np.abs(ref).max())
            k += 1
    assert k == d.shape[0]
    # the tables are the same with or without the Delta output
    la2, ar2, ep2 = ctx.pair_eval()
    assert torch.equal(la, la2) and torch.equal(ep, ep2)
    ctx.close()
