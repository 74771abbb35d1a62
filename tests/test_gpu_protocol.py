"""Rank-growing protocol of Sec. III.C through the C ABI: sgs_rotate against
numpy, and the whole protocol (steps at rank 1, then one rotated copy of the
largest-amplitude state per rank) against the oracle's ``grow`` with the same
seeded rotations.  Tolerances: the rotation is two float64 products
(1e-13 absolute); the trajectories as the Euler trajectory test (1e-10
relative on the energies)."""

import sys

import numpy as np
import pytest

import sgs_inputs as si
from oracle import sgs as osgs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("n", [12, 132])
def test_rotate_matches_numpy(n):
    from paper_2105_01088_amd import rotate_state
    _say(f"[grow] rotate n={n}")
    g = si.random_states(n // 2, 1, seed=2)[0]
    Q = si.small_rotations(n, 1, 0.3, seed=4)[0]
    out = rotate_state(torch.as_tensor(Q, device="cuda"), torch.as_tensor(g, device="cuda")).cpu().numpy()
    ref = Q @ g @ Q.T
    assert np.abs(out - ref).max() < 1e-13
    assert np.abs(out + out.T).max() == 0.0
    assert np.abs(out @ out + np.eye(n)).max() < 1e-12


@pytest.mark.parametrize("L,nrot,steps", [(2, 2, 40), (7, 3, 15)])
def test_grow_matches_oracle(L, nrot, steps):
    from paper_2105_01088_amd import default_options, grow
    N, terms = si.anderson_terms(L, 1.3, 0.7)
    ham = si.MajoranaHamiltonian.from_poly(N, si.fermion_terms_to_majorana(terms))
    g0 = si.random_states(ham.N, 1, seed=3)[0]
    rots = si.small_rotations(ham.n, nrot, 0.3, seed=1)
    _say(f"[grow] anderson L={L} n={ham.n} ranks 1..{nrot + 1}, {steps} steps each")
    g, e, ranks = grow(ham, g0, 0.05, steps, rots, options=default_options(weight=1))
    e = e.cpu().numpy()
    gr, er, rr = osgs.grow(ham, g0, 0.05, steps, rots, mode="unit")
    assert ranks == rr and g.shape[0] == nrot + 1
    assert np.abs(e - er).max() < 1e-10 * np.abs(er).max()
    assert np.abs(g.cpu().numpy() - gr).max() < 1e-8
