"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Tolerances (float64 path): the pair inverse and the Pfaffian lose about
kappa * n * eps relative accuracy (kappa = cond(Gamma_a + Gamma_b), a few
hundred to a few thousand for the seeded random states used here), so tables
are compared at 1e-9 (log|G|, phase, eps), one-step covariance matrices at
1e-10 absolute and energies at 1e-10 relative.

With the printed weights c_mu = 1 / (lambda_mu lambda~_mu^*) the force on
state mu carries lambda_b / lambda_mu: the eigenvector's error (bounded by
the eigen-solver's backward error) becomes a relative error of order
delta / |lambda_mu| in that force.  Random states are nearly orthogonal and
some amplitudes are tiny, so for that mode each state's covariance tolerance
adds its own bound (tests/parity_tol.py).
"""

import math
import sys

import numpy as np
import pytest

import sgs_inputs as si
from oracle import sgs as osgs
from parity_tol import phase_tol, printed_tol

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_TAB = 1e-9
TOL_GAMMA = 1e-10
TOL_E = 1e-10


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _ctx(ham, gam, weight=0, **kw):
    from paper_2105_01088_amd import SGS, default_options
    return SGS([ham], [gam], options=default_options(weight=weight, **kw))


def _tables(ctx):
    la, ar, ep = ctx.pair_eval()
    assert ctx.status() == 0
    R = ctx.R[0]
    la = la.cpu().numpy().reshape(R, R)
    ar = ar.cpu().numpy().reshape(R, R)
    ep = ep.cpu().numpy().reshape(R, R, 2)
    return la, ar, ep[..., 0] + 1j * ep[..., 1]


def _cmp_tables(ham, gam, tag):
    _say(f"[pair_eval] {tag} n={gam.shape[1]} R={gam.shape[0]}")
    ctx = _ctx(ham, gam)
    la, ar, ep = _tables(ctx)
    ref = osgs.pair_tables(ham, gam)
    R = gam.shape[0]
    off = ~np.eye(R, dtype=bool)
    if R > 1:
        assert np.abs(la - ref.logabs)[off].max() < TOL_TAB * max(1.0, np.abs(ref.logabs).max())
        assert np.abs(np.exp(1j * ar) - np.exp(1j * ref.arg)).max() < TOL_TAB
    scale = max(1.0, np.abs(ref.eps).max())
    assert np.abs(ep - ref.eps).max() < TOL_TAB * scale
    ctx.close()


@pytest.mark.parametrize("L,R,seed", [(3, 4, 1), (24, 5, 2), (32, 6, 3)])
def test_pair_tables_anderson(L, R, seed):
    ham = si.anderson(L, 1.3, 0.6)
    gam = si.random_states(ham.N, R, seed)
    _cmp_tables(ham, gam, f"anderson L={L}")


def test_pair_tables_two_channel_kondo():
    ham = si.two_channel_kondo(3, 0.5, U=8.0)
    gam = si.random_states(ham.N, 4, 5)
    _cmp_tables(ham, gam, "tck L=3")


@pytest.mark.parametrize("weight", [0, 1])
@pytest.mark.parametrize("L,R,seed", [(1, 3, 3), (3, 4, 1), (32, 3, 7)])
def test_one_step_matches_oracle(weight, L, R, seed):
    ham = si.anderson(L, 1.3, 0.6)
    gam = si.random_states(ham.N, R, seed)
    _say(f"[step] anderson L={L} R={R} weight={weight}")
    ctx = _ctx(ham, gam, weight=weight)
    e = ctx.step(0.05, 1)
    assert ctx.status() == 0
    g_new = ctx.gammas(0).cpu().numpy()
    ref = osgs.step(ham, gam, 0.05, mode="printed" if weight == 0 else "unit")
    assert abs(e.cpu().item() - ref.E) < TOL_E * abs(ref.E)
    err = np.abs(g_new - ref.gammas)
    tol = _gamma_tol(ref, weight, 0.05)
    _say(f"  err {err.max():.2e}, tol {np.min(tol):.2e}..{np.max(tol):.2e}")
    assert np.all(err < tol)
    ctx.close()


def _gamma_tol(ref, weight, dtau):
    """1e-10, and for printed weights the per-state bound of parity_tol."""
    if weight != 0:
        return TOL_GAMMA
    return printed_tol(ref, dtau, TOL_GAMMA)[0][:, None, None]


@pytest.mark.parametrize("R", [1, 2])
def test_small_rank_edge_cases(R):
    ham = si.anderson(5, 1.0, 0.5)
    gam = si.random_states(ham.N, R, 11)
    _say(f"[step] edge R={R}")
    ctx = _ctx(ham, gam)
    e = ctx.step(0.05, 2)
    assert ctx.status() == 0
    g = gam
    es = []
    for _ in range(2):
        r = osgs.step(ham, g, 0.05)
        es.append(r.E)
        g = r.gammas
    assert np.allclose(e.cpu().numpy(), es, rtol=TOL_E, atol=0)
    assert np.abs(ctx.gammas(0).cpu().numpy() - g).max() < TOL_GAMMA
    ctx.close()


def _tiny_ham(N, seed, quartic):
    rng = np.random.default_rng(seed)
    n = 2 * N
    z = rng.standard_normal((n, n))
    qi = np.array([[0, 1, 2, 3]], dtype=np.int32) if quartic else np.zeros((0, 4), dtype=np.int32)
    qv = np.array([0.6]) if quartic else np.zeros(0)
    return si.MajoranaHamiltonian(N=N, A=0.5 * (z - z.T), quartic_idx=qi, quartic_val=qv, e0=0.1)


@pytest.mark.parametrize("N,R", [(2, 1), (2, 2), (2, 3), (2, 4), (1, 1), (1, 2)])
def test_tiny_systems(N, R):
    """The degenerate sizes: two modes (n = 4, one quartic word; the even
    sector has dimension 2, so R >= 2 is exact and R = 3, 4 leave G
    singular) and one mode (n = 2: every pure even state is the same one,
    so R = 2 gives two identical states).  Matrices narrower than every
    panel and tile, Pfaffians of order 2, canonical orthogonalization
    dropping vectors; two steps at 1e-10."""
    ham = _tiny_ham(N, N, N == 2)
    gam = si.random_states(N, R, 3 + R)
    _say(f"[step] tiny n={ham.n} R={R}")
    ctx = _ctx(ham, gam, weight=1)
    e = ctx.step(0.05, 2).cpu().numpy().ravel()
    assert ctx.status() == 0
    g = gam
    es = []
    for _ in range(2):
        r = osgs.step(ham, g, 0.05, mode="unit")
        es.append(r.E)
        g = r.gammas
    assert np.abs(e - es).max() < TOL_E * max(1.0, np.abs(es).max())
    assert np.abs(ctx.gammas(0).cpu().numpy() - g).max() < TOL_GAMMA
    ctx.close()


def test_two_channel_kondo_step():
    ham = si.two_channel_kondo(3, 0.5, U=8.0)
    gam = si.random_states(ham.N, 3, 2)
    _say("[step] tck L=3 R=3")
    ctx = _ctx(ham, gam)
    e = ctx.step(0.05, 1)
    assert ctx.status() == 0
    ref = osgs.step(ham, gam, 0.05)
    assert abs(e.cpu().item() - ref.E) < TOL_E * abs(ref.E)
    assert np.abs(ctx.gammas(0).cpu().numpy() - ref.gammas).max() < TOL_GAMMA
    ctx.close()


def test_anderson_L7_trajectory_and_bounds():
    import json
    import os
    ham, gam, cfg = si.config_problem("anderson_L7_R4")
    _say("[trajectory] anderson L=7 R=4, 20 steps")
    ctx = _ctx(ham, gam)
    e = ctx.step(0.05, 20).cpu().numpy()
    assert ctx.status() == 0
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "anderson_L7.json")))
    first10 = np.array(gold["anderson_L7_R4_seed0_first10_E"]["value"])
    assert np.abs(e[:10] - first10).max() < TOL_E * np.abs(first10).max()
    _, es = osgs.run(ham, gam, 0.05, 20)
    assert np.abs(e - es).max() < TOL_E * np.abs(es).max()
    e_ed = gold["anderson_L7_U1_V0.5_ed_even"]["value"]
    assert np.all(e >= e_ed - 1e-12)
    assert np.all(np.diff(e) <= 1e-12)
    g = ctx.gammas(0).cpu().numpy()
    for x in g:
        assert np.abs(x + x.T).max() == 0.0
        assert np.abs(x @ x + np.eye(x.shape[0])).max() < 1e-12
    ctx.close()


# ---------------------------------------------------------------- full sizes

def test_anderson_L99_R16_one_step():
    """The benchmark workload (n = 400, R = 16), in the launch configuration
    bench.py times, one step against the oracle."""
    ham, gam, cfg = si.config_problem("anderson_L99_R16")
    _say("[step] anderson_L99_R16 (n=400, R=16), unit weights")
    ctx = _ctx(ham, gam, weight=1)
    e = ctx.step(0.05, 1)
    assert ctx.status() == 0
    g_new = ctx.gammas(0).cpu().numpy()
    ref = osgs.step(ham, gam, 0.05, mode="unit")
    assert abs(e.cpu().item() - ref.E) < TOL_E * abs(ref.E)
    assert np.abs(g_new - ref.gammas).max() < TOL_GAMMA
    ctx.close()


def _sampled_tables(name, pairs, phase_pairs):
    from oracle import gaussian as ga
    ham, gam, cfg = si.config_problem(name)
    R = gam.shape[0]
    _say(f"[pair_eval] {name} (n={ham.n}, R={R}), sampled pairs")
    ctx = _ctx(ham, gam, weight=1)
    la, ar, ep = _tables(ctx)
    hp = ham.poly()
    for a, b in pairs:
        ref = ga.log_abs_overlap(gam[a], gam[b])
        assert abs(la[a, b] - ref) < TOL_TAB * abs(ref)
        assert la[b, a] == la[a, b]
        d = ga.delta(gam[b], gam[a])  # Delta^{ba}: eps_ab
        e_ref = ga.poly_value(d, hp)
        assert abs(ep[a, b] - e_ref) < TOL_TAB * max(1.0, abs(e_ref))
    g0 = gam[0]
    for a, b in phase_pairs:
        _, ph = ga.triple_product_schur(g0, gam[a], gam[b])
        tol = phase_tol(g0, gam[a], gam[b])
        err = abs(np.exp(1j * ar[a, b]) - ph)
        _say(f"  phase ({a}, {b}): error {err:.3g}, tolerance {tol:.3g}")
        assert err < tol
        assert abs(ar[b, a] + ar[a, b]) < 1e-15
    for a in range(R):
        assert ar[0, a] == 0.0
    ctx.close()


def test_anderson_L199_R32_sampled_tables():
    _sampled_tables("anderson_L199_R32_U1", [(0, 1), (3, 17), (30, 31)], [(1, 2), (5, 29), (30, 31)])


def test_two_channel_kondo_L150_R24_sampled_tables():
    _sampled_tables("tck_L150_R24_J0.3", [(0, 23), (7, 8)], [(1, 23), (11, 12)])


# ------------------------------------------------------------- FP32 path

def _run(ham, gam, steps, **kw):
    ctx = _ctx(ham, gam, **kw)
    e = ctx.step(0.05, steps).cpu().numpy()
    assert ctx.status() == 0
    g = ctx.gammas(0).cpu().numpy()
    ctx.close()
    return e, g


def test_fp32_one_step_against_oracle():
    """FP32 path: the energy entering the step is the float64 one; the new
    covariance matrices differ from the oracle's by the float32 rounding of
    the force product: at most 1e-5 dtau max|dGamma| here (float32 epsilon
    6e-8 times K = 2 n R = 360 products, allowing for cancellation)."""
    ham = si.anderson(8, 1.3, 0.6)
    gam = si.random_states(ham.N, 5, 9)
    _say("[fp32] anderson L=8 R=5")
    e, g = _run(ham, gam, 1, weight=1, precision=1)
    ref = osgs.step(ham, gam, 0.05, mode="unit")
    assert abs(e[0] - ref.E) < TOL_E * abs(ref.E)
    err = np.abs(g - ref.gammas).max()
    assert err < 1e-5 * 0.05 * np.abs(ref.dgamma).max()
    assert err > 0.0  # the float product is really used


def test_fp32_plain_error_bound():
    """FP32 path at the benchmark size: after 5 steps the states and energies
    follow the float64 run closely, and the energy still decreases."""
    ham, gam, cfg = si.config_problem("anderson_L99_R16")
    _say("[fp32] anderson_L99_R16, 5 steps against float64")
    e64, g64 = _run(ham, gam, 5, weight=1)
    e32, g32 = _run(ham, gam, 5, weight=1, precision=1)
    assert e32[0] == e64[0]  # the first energy does not see the force
    assert np.abs(g32 - g64).max() < 1e-5
    assert np.abs(e32 - e64).max() < 1e-8 * np.abs(e64).max()
    assert np.all(np.diff(e32) <= 1e-10 * abs(e32[0]))


@pytest.mark.parametrize("tile", [64, 128])
@pytest.mark.parametrize("L,R,seed", [(32, 3, 5), (64, 4, 6)])
def test_force_tiles_match_oracle(tile, L, R, seed):
    """Both force tile edges (64 x 64, 128 x 128 with eight waves) on ragged
    sizes n = 132 and 260 (one tile plus a sliver; two plus a sliver),
    whatever the built-in choice for that n: one step at 1e-10.  Rotated
    near-copy states give overlaps of order one, so the cross terms and the
    complex coefficients weigh as much as the self terms (with seeded random
    states they are negligible)."""
    ham = si.anderson(L, 1.2, 0.7)
    gam = si.near_copy_states(ham.N, R, 1.5, seed=seed)
    _say(f"[step] force tile {tile}, n={ham.n} R={R}")
    ctx = _ctx(ham, gam, weight=1, tune=[{"n_max": 4096, "force_tile": tile}])
    e = ctx.step(0.05, 1)
    assert ctx.status() == 0
    g_new = ctx.gammas(0).cpu().numpy()
    ref = osgs.step(ham, gam, 0.05, mode="unit")
    assert abs(e.cpu().item() - ref.E) < TOL_E * abs(ref.E)
    assert np.abs(g_new - ref.gammas).max() < TOL_GAMMA
    ctx.close()


@pytest.mark.parametrize("row", [
    {"gj_super": 32}, {"gj_super": 96}, {"gj_super": 256},
    {"gj_first": 1}, {"gj_first": 2},
    {"pf_super": 1}, {"pf_super": 8}, {"pf_super": 24}, {"pf_super": 32},
    {"force_split": 1}, {"force_split": 3}, {"force_elem": 2},
    {"gj_super": 64, "gj_defer": 3, "pf_super": 24, "force_split": 2, "force_elem": 2},
])
def test_tuning_choices_match_oracle(row):
    """Every scheduling and blocking choice a tuning row can make (the
    autotuner may pick any of them) leaves the results those of the oracle:
    Gauss-Jordan super-panels of one panel up to 256 columns, the order of
    the two inverse batches, Pfaffian super-panels of 1 to 32 steps (ragged
    against the 16-step register panels), the force's term split and the
    elementwise terms on either stream; n = 260 (two panels plus a sliver),
    rotated near-copy states.  Pair tables at 1e-9, one step at 1e-10."""
    ham = si.anderson(64, 1.1, 0.6)
    gam = si.near_copy_states(ham.N, 4, 1.5, seed=21)
    _say(f"[step] tuning {row}, n={ham.n} R=4")
    ctx = _ctx(ham, gam, weight=1, tune=[dict(n_max=4096, **row)])
    la, ar, ep = _tables(ctx)
    tab = osgs.pair_tables(ham, gam)
    off = ~np.eye(4, dtype=bool)
    assert np.abs(la - tab.logabs)[off].max() < TOL_TAB * max(1.0, np.abs(tab.logabs).max())
    assert np.abs(np.exp(1j * ar) - np.exp(1j * tab.arg))[off].max() < TOL_TAB
    assert np.abs(ep - tab.eps).max() < TOL_TAB * max(1.0, np.abs(tab.eps).max())
    e = ctx.step(0.05, 1)
    assert ctx.status() == 0
    g_new = ctx.gammas(0).cpu().numpy()
    ref = osgs.step(ham, gam, 0.05, mode="unit")
    assert abs(e.cpu().item() - ref.E) < TOL_E * abs(ref.E)
    assert np.abs(g_new - ref.gammas).max() < TOL_GAMMA
    ctx.close()


@pytest.mark.parametrize("defer", [1, 2, 3])
@pytest.mark.parametrize("L,R,seed", [(32, 5, 5), (64, 4, 6), (99, 5, 7)])
def test_gj_deferral_matches_oracle(defer, L, R, seed):
    """The Gauss-Jordan inner updates applied after every panel (1), deferred
    for the pairs not involving state 0 (2) or for all pairs (3), on n = 132,
    260 and 400 (super-panels of 128 plus a ragged one), whatever the built-in
    choice: the pair tables at 1e-9 and one step at 1e-10."""
    ham = si.anderson(L, 1.2, 0.7)
    gam = si.random_states(ham.N, R, seed)
    _say(f"[step] gj_defer {defer}, n={ham.n} R={R}")
    ctx = _ctx(ham, gam, weight=1, tune=[{"n_max": 4096, "gj_defer": defer}])
    la, ar, ep = _tables(ctx)
    tab = osgs.pair_tables(ham, gam)
    off = ~np.eye(R, dtype=bool)
    assert np.abs(la - tab.logabs)[off].max() < TOL_TAB * max(1.0, np.abs(tab.logabs).max())
    assert np.abs(ep - tab.eps).max() < TOL_TAB * max(1.0, np.abs(tab.eps).max())
    e = ctx.step(0.05, 1)
    assert ctx.status() == 0
    g_new = ctx.gammas(0).cpu().numpy()
    ref = osgs.step(ham, gam, 0.05, mode="unit")
    assert abs(e.cpu().item() - ref.E) < TOL_E * abs(ref.E)
    assert np.abs(g_new - ref.gammas).max() < TOL_GAMMA
    ctx.close()
