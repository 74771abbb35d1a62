"""The allocation-free entry point sgs_rotate_noalloc (fixed device scratch
instead of a work buffer) against sgs_rotate, through the C ABI.

Two calls in a row on one device, the second with a smaller n, so the second
reuses the scratch the first left behind; the kernels are the same, so the
results must agree bit for bit.  A size above the scratch is refused on the
host with SGS_ESCRATCH before any GPU work."""

import sys

import numpy as np
import pytest

import sgs_inputs as si

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case(n, seed):
    rng = np.random.default_rng(seed)
    Q = si.small_rotations(n, 1, 0.3, seed=seed)[0]
    g = si.random_states(n // 2, 1, seed=seed)[0]
    return (torch.tensor(Q, device="cuda:0"), torch.tensor(g, device="cuda:0"))


def test_noalloc_rotate_matches_rotate_twice():
    from paper_2105_01088_amd import rotate_state, rotate_state_noalloc
    for n, seed in ((1204, 3), (400, 4)):
        print(f"[noalloc] sgs_rotate_noalloc n={n} seed={seed}", flush=True)
        Q, g = _case(n, seed)
        ref = rotate_state(Q, g)
        got = rotate_state_noalloc(Q, g)
        torch.cuda.synchronize()
        ref = ref.cpu().numpy()
        got = got.cpu().numpy()
        assert np.array_equal(got, ref)
        # and against numpy (same product, rounding order aside)
        qn, gn = Q.cpu().numpy(), g.cpu().numpy()
        want = qn @ gn @ qn.T
        want = 0.5 * (want - want.T)
        assert np.abs(got - want).max() < 1e-12 * n


def test_noalloc_rotate_rejects_sizes_above_scratch():
    from paper_2105_01088_amd import load_library
    lib = load_library()
    print("[noalloc] n=1538 refused", flush=True)
    x = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    rc = lib.sgs_rotate_noalloc(x.data_ptr(), x.data_ptr(), x.data_ptr(), 1538, None)
    assert rc == -11  # SGS_ESCRATCH, returned before any launch
    rc = lib.sgs_rotate_noalloc(x.data_ptr(), x.data_ptr(), x.data_ptr(), 7, None)
    assert rc == -1  # odd n: SGS_EINVAL
