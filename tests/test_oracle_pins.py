"""Pins of the CPU oracle against facts fixed outside it.

Every check here compares the oracle with something it does not compute itself:
brute-force Fock-space vectors (Jordan-Wigner), the defining Pfaffian
expansion, closed forms, exact diagonalization and invariants stated in the
paper.  A wrong sign, dropped term, swapped index or transposed operand in the
oracle fails at least one of them.
"""

import math

import numpy as np
import pytest

import sgs_inputs as si
from oracle import ed, fock, gaussian as ga, observables as ob, sgs
from oracle.pfaffian import pfaffian, pfaffian_expand, pfaffian_log


def _rand_skew(n, rng, cplx=False):
    a = rng.standard_normal((n, n))
    if cplx:
        a = a + 1j * rng.standard_normal((n, n))
    return a - a.T


# ----------------------------------------------------------------- Pfaffian

@pytest.mark.parametrize("n", [2, 4, 6, 8])
@pytest.mark.parametrize("cplx", [False, True])
def test_pfaffian_matches_expansion(n, cplx):
    rng = np.random.default_rng(n + 10 * cplx)
    a = _rand_skew(n, rng, cplx)
    assert abs(pfaffian(a) - pfaffian_expand(a)) < 1e-12 * max(1.0, abs(pfaffian_expand(a)))


@pytest.mark.parametrize("n", [10, 40])
def test_pfaffian_square_is_det_and_congruence(n):
    rng = np.random.default_rng(n)
    a = _rand_skew(n, rng, True)
    p = pfaffian(a)
    assert abs(p * p - np.linalg.det(a)) < 1e-9 * abs(p * p)
    q = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    p2 = pfaffian(q.T @ a @ q)
    assert abs(p2 - np.linalg.det(q) * p) < 1e-8 * abs(p2)


def test_pfaffian_canonical_block_form():
    # Pf of (+) [[0, a_j], [-a_j, 0]] is prod a_j; a basis swap flips the sign
    a = np.array([0.5, -2.0, 3.0])
    m = np.zeros((6, 6))
    for j, x in enumerate(a):
        m[2 * j, 2 * j + 1], m[2 * j + 1, 2 * j] = x, -x
    assert abs(pfaffian(m) - np.prod(a)) < 1e-14
    perm = [1, 0, 2, 3, 4, 5]
    assert abs(pfaffian(m[np.ix_(perm, perm)]) + np.prod(a)) < 1e-14
    assert pfaffian_log(np.zeros((4, 4)))[0] == -math.inf


# ------------------------------------------------------- models and states

@pytest.mark.parametrize("builder", [
    lambda: si.anderson_terms(1, 1.3, 0.7),
    lambda: si.anderson_terms(2, 2.0, 0.4, t=0.8, mu=0.1),
    lambda: si.two_channel_kondo_terms(1, 0.7, U=3.0),
])
def test_majorana_form_equals_fermionic_operator(builder):
    N, terms = builder()
    poly = si.fermion_terms_to_majorana(terms)
    ham = si.MajoranaHamiltonian.from_poly(N, poly)
    hm = fock.majorana_poly_operator(N, ham.poly())
    hf = fock.fermion_operator(N, terms)
    assert np.abs(hm - hf).max() < 1e-13


def test_anderson_closed_form_coefficients():
    # -t (a_j^dag a_k + h.c.) -> A[2j, 2k+1] = -t/4, A[2j+1, 2k] = t/4;
    # U n_up n_dn at eps_d = -U/2 -> no impurity quadratic term, e0 = -U/4, u = -U/4
    h = si.anderson(3, 2.0, 0.6)
    assert h.A[0, 5] == pytest.approx(-0.6 / 4) and h.A[1, 4] == pytest.approx(0.6 / 4)
    assert h.A[4, 9] == pytest.approx(-0.25) and h.A[5, 8] == pytest.approx(0.25)
    assert h.A[0, 1] == 0.0 and h.A[2, 3] == 0.0
    assert h.e0 == pytest.approx(-0.5)
    assert h.quartic_idx.tolist() == [[0, 1, 2, 3]] and h.quartic_val[0] == pytest.approx(-0.5)
    assert np.abs(h.A + h.A.T).max() == 0.0


def test_two_channel_kondo_structure():
    h = si.two_channel_kondo(150, 0.3)
    assert h.N == 602 and h.n == 1204
    assert len(h.quartic_val) == 25
    assert sorted(set(np.round(np.abs(h.quartic_val[1:]), 12))) == [round(0.3 / 16, 12)]
    assert len(h.impurity_majoranas()) == 12


def test_spin_dot_poly_equals_fermionic():
    N = 4
    poly = si.spin_dot_poly((0, 1), (2, 3))
    hm = fock.majorana_poly_operator(N, poly)
    hf = fock.fermion_operator(N, si.spin_dot_terms((0, 1), (2, 3)))
    assert np.abs(hm - hf).max() < 1e-14


def test_random_states_pure_even_and_vacuum_convention():
    g = si.random_states(4, 3, seed=7)
    for x in g:
        assert np.abs(x + x.T).max() == 0.0
        assert np.abs(x @ x + np.eye(8)).max() < 1e-13
        assert pfaffian(x) == pytest.approx(1.0, abs=1e-12)
    vac = np.zeros(2 ** 4)
    vac[0] = 1.0
    assert np.abs(fock.covariance(vac, 4) - si.vacuum_cm(4)).max() < 1e-15
    for x in g:
        psi = fock.gaussian_state(x)
        assert np.abs(fock.covariance(psi, 4) - x).max() < 1e-12
        par = np.vdot(psi, fock.parity_operator(4) @ psi).real
        assert par == pytest.approx(1.0, abs=1e-12)


# -------------------------------------------------------- overlaps and Wick

@pytest.fixture(scope="module")
def tiny():
    ham = si.anderson(1, 1.3, 0.7)
    g = si.random_states(ham.N, 3, seed=3)
    vecs = [fock.gaussian_state(x) for x in g]
    vecs = fock.fix_gauge(vecs, vecs[0])
    return ham, g, vecs


def test_overlap_magnitude_and_pfaffian_sign(tiny):
    ham, g, vecs = tiny
    N = ham.N
    for a in range(3):
        for b in range(3):
            if a == b:
                continue
            ov = abs(np.vdot(vecs[a], vecs[b]))
            assert math.exp(ga.log_abs_overlap(g[a], g[b])) == pytest.approx(ov, rel=1e-12)
            # same-parity states: Pf(G_a + G_b) = 2^N |<a|b>|^2 >= 0 (no sign ambiguity)
            assert pfaffian(g[a] + g[b]) == pytest.approx(2 ** N * ov ** 2, rel=1e-12)


@pytest.mark.parametrize("direct", [False, True])
def test_triple_product_phase(tiny, direct):
    ham, g, vecs = tiny
    t = np.vdot(vecs[0], vecs[1]) * np.vdot(vecs[1], vecs[2]) * np.vdot(vecs[2], vecs[0])
    f = ga.triple_product_direct if direct else ga.triple_product_schur
    la, ph = f(g[0], g[1], g[2])
    assert abs(ph * math.exp(la) - t) < 1e-13


def test_gram_matrix_in_reference_gauge(tiny):
    ham, g, vecs = tiny
    V = np.stack(vecs, 1)
    assert np.abs(ga.gram(g) - V.conj().T @ V).max() < 1e-13
    assert np.abs(ga.gram(g, use_direct=True) - V.conj().T @ V).max() < 1e-13


def test_transition_matrix(tiny):
    ham, g, vecs = tiny
    N, n = ham.N, ham.n
    c = fock.majoranas(N)
    for a, b in [(1, 2), (2, 0), (0, 1)]:
        d = ga.delta(g[a], g[b])
        gba = np.vdot(vecs[b], vecs[a])
        for k in range(n):
            for l in range(n):
                if k != l:
                    v = np.vdot(vecs[b], c[k] @ c[l] @ vecs[a])
                    assert abs(v - 1j * gba * d[k, l]) < 1e-13
        assert np.abs(d + d.T).max() < 1e-12                         # skew
        assert np.abs(d - ga.delta(g[b], g[a]).conj()).max() < 1e-12  # D^{ab} = conj D^{ba}
        assert np.abs(d @ d + np.eye(n)).max() < 1e-11               # D^2 = -1
    assert np.abs(ga.delta(g[1], g[1]) - g[1]).max() < 1e-13          # D^{aa} = Gamma_a


@pytest.mark.parametrize("model", ["anderson", "tck"])
def test_projected_hamiltonian(model):
    if model == "anderson":
        N, terms = si.anderson_terms(1, 1.3, 0.7)
    else:
        N, terms = si.two_channel_kondo_terms(1, 0.9, U=2.0)
    ham = si.MajoranaHamiltonian.from_poly(N, si.fermion_terms_to_majorana(terms))
    g = si.random_states(N, 3, seed=11)
    vecs = fock.fix_gauge([fock.gaussian_state(x) for x in g], fock.gaussian_state(g[0]))
    vecs = fock.fix_gauge(vecs, vecs[0])
    V = np.stack(vecs, 1)
    H = fock.fermion_operator(N, terms)
    tab = sgs.pair_tables(ham, g)
    assert np.abs(tab.G - V.conj().T @ V).max() < 1e-13
    assert np.abs(tab.h - V.conj().T @ H @ V).max() < 1e-12


# ------------------------------------------------------------------- force

def _bruteforce_force(ham, g, mode):
    N, n, R = ham.N, ham.n, g.shape[0]
    vecs = fock.fix_gauge([fock.gaussian_state(x) for x in g], fock.gaussian_state(g[0]))
    vecs = fock.fix_gauge(vecs, vecs[0])
    V = np.stack(vecs, 1)
    H = fock.majorana_poly_operator(N, ham.poly())
    Gb, hb = V.conj().T @ V, V.conj().T @ H @ V
    E, lam = sgs.solve_amplitudes(Gb, hb)
    psi = V @ lam
    lamt = Gb @ lam
    c = sgs.weights(lam, lamt, mode)
    pperp = np.eye(2 ** N) - V @ np.linalg.inv(Gb) @ V.conj().T  # projector of Eq. (projImEvol)
    cm = fock.majoranas(N)
    out = np.zeros((R, n, n))
    for mu in range(R):
        B = c[mu] * np.outer(pperp @ H @ psi, psi.conj())       # Eq. (Bmu)
        B = B + B.conj().T
        dphi = -B @ vecs[mu]                                     # Eq. (PhiMu)
        for k in range(n):
            for l in range(n):
                if k != l:
                    v = -1j * np.vdot(vecs[mu], cm[k] @ cm[l] @ dphi)
                    out[mu, k, l] = 2 * v.real
    return out


@pytest.mark.parametrize("mode", ["printed", "unit"])
@pytest.mark.parametrize("model", ["anderson", "tck"])
def test_force_matches_bruteforce_derivative(mode, model):
    if model == "anderson":
        ham = si.anderson(1, 1.3, 0.7)
    else:
        ham = si.two_channel_kondo(1, 0.9, U=2.0)
    g = si.random_states(ham.N, 3, seed=3)
    tab = sgs.pair_tables(ham, g)
    E, lam = sgs.solve_amplitudes(tab.G, tab.h)
    dg = sgs.forces(ham, g, tab, E, lam, mode)
    ref = _bruteforce_force(ham, g, mode)
    assert np.abs(dg - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())
    for mu in range(3):  # purity preservation, Sec. III.B
        assert np.abs(dg[mu] @ g[mu] + g[mu] @ dg[mu]).max() < 1e-12


def _fock_setup(ham, g):
    N = ham.N
    vecs = fock.fix_gauge([fock.gaussian_state(x) for x in g], fock.gaussian_state(g[0]))
    vecs = fock.fix_gauge(vecs, vecs[0])
    V = np.stack(vecs, 1)
    H = fock.majorana_poly_operator(N, ham.poly())
    return vecs, V, H


@pytest.mark.parametrize("mode", ["printed", "unit"])
def test_weights_satisfy_the_descent_condition(mode):
    """Sec. III.A: the weight makes every state descend, c_mu lambda~_mu^*
    lambda_mu real and positive; the unit-modulus choice has |c_mu| = 1; with
    the printed choice the states move together as Eq. (projImEvol2) asks,
    sum_mu lambda_mu |dphi_mu> = -R Pi_perp H |psi> (R times the printed
    right-hand side: each of the R states carries the full projected step).
    Checked in Fock space, independently of how sgs.weights is written."""
    ham = si.anderson(1, 1.1, 0.6)
    g = si.random_states(ham.N, 3, seed=21)
    vecs, V, H = _fock_setup(ham, g)
    Gb, hb = V.conj().T @ V, V.conj().T @ H @ V
    E, lam = sgs.solve_amplitudes(Gb, hb)
    lamt = Gb @ lam
    c = sgs.weights(lam, lamt, mode)
    d = c * lamt.conj() * lam
    assert np.all(d.real > 0) and np.abs(d.imag).max() < 1e-12 * np.abs(d).max()
    if mode == "unit":
        assert np.allclose(np.abs(c), 1.0, atol=1e-14, rtol=0)
    else:
        psi = V @ lam
        pperp = np.eye(V.shape[0]) - V @ np.linalg.inv(Gb) @ V.conj().T
        target = -3 * (pperp @ H @ psi)
        tot = np.zeros_like(psi)
        for mu in range(3):
            B = c[mu] * np.outer(pperp @ H @ psi, psi.conj())   # Eq. (Bmu)
            B = B + B.conj().T
            tot += lam[mu] * (-B @ vecs[mu])                      # Eq. (PhiMu)
        assert np.abs(tot - target).max() < 1e-12 * np.abs(target).max()


def test_force_with_dropped_combination_matches_bruteforce():
    """Two states differ by a rotation of |Q - 1|_F = 1e-7: G has an eigenvalue
    below 1e-12 of its largest, which canonical orthogonalization drops.  The
    long form of Eq. (EOM-Gamma3) with G^-1 read as the inverse on the kept
    subspace equals the brute-force derivative with the projector onto the
    complement of the kept combinations (and differs from it at O(1) with the
    plain G^-1, so a dropped term or the wrong inverse fails here)."""
    ham = si.anderson(1, 1.2, 0.5)
    g0 = si.random_states(ham.N, 2, seed=8)
    q = si.small_rotations(ham.n, 1, 1e-7, seed=9)[0]
    g2 = q @ g0[1] @ q.T
    g = np.stack([g0[0], g0[1], 0.5 * (g2 - g2.T)])
    tab = sgs.pair_tables(ham, g)
    X = sgs.canonical_basis(tab.G)
    assert X.shape[1] == 2  # one combination dropped
    E, lam = sgs.solve_amplitudes(tab.G, tab.h)
    for mode in ("printed", "unit"):
        dg = sgs.forces(ham, g, tab, E, lam, mode)
        vecs, V, H = _fock_setup(ham, g)
        Gb = V.conj().T @ V
        lamt = Gb @ lam
        c = sgs.weights(lam, lamt, mode)
        VX = V @ X
        pperp = np.eye(V.shape[0]) - VX @ VX.conj().T
        psi = V @ lam
        cm = fock.majoranas(ham.N)
        for mu in range(3):
            B = c[mu] * np.outer(pperp @ H @ psi, psi.conj())
            B = B + B.conj().T
            dphi = -B @ vecs[mu]
            ref = np.zeros((ham.n, ham.n))
            for k in range(ham.n):
                for l in range(ham.n):
                    if k != l:
                        ref[k, l] = 2 * (-1j * np.vdot(vecs[mu], cm[k] @ cm[l] @ dphi)).real
            # the kept combinations mix two vectors that differ by 1e-7, so
            # float64 rounding (1e-16) in either side is magnified ~1e7
            assert np.abs(dg[mu] - ref).max() < 1e-7 * max(1.0, np.abs(ref).max())


def test_rank_one_is_ghf_imaginary_time():
    # R = 1: the normalization line cancels and dGamma = 4 (F + Gamma F Gamma)
    ham = si.anderson(2, 1.5, 0.6)
    g = si.random_states(ham.N, 1, seed=2)
    tab = sgs.pair_tables(ham, g)
    E, lam = sgs.solve_amplitudes(tab.G, tab.h)
    dg = sgs.forces(ham, g, tab, E, lam, "printed")
    F = ga.fock_matrix(ham, g[0]).real
    assert np.abs(dg[0] - 4 * (F + g[0] @ F @ g[0])).max() < 1e-12


def test_purify_is_canonical_form_rescaling():
    rng = np.random.default_rng(0)
    g = si.random_states(5, 1, seed=1)[0]
    x = g + 0.05 * _rand_skew(10, rng)
    p = sgs.purify(x)
    assert np.abs(p @ p + np.eye(10)).max() < 1e-13
    # polar factor: p^T x is symmetric positive definite
    s = p.T @ x
    assert np.abs(s - s.T).max() < 1e-12 and np.linalg.eigvalsh(0.5 * (s + s.T)).min() > 0


def test_reference_state_choice_does_not_change_physics():
    ham = si.anderson(1, 1.3, 0.7)
    g = si.random_states(ham.N, 3, seed=4)
    r1 = sgs.step(ham, g, 0.05)
    perm = [2, 0, 1]
    r2 = sgs.step(ham, g[perm], 0.05)
    assert r1.E == pytest.approx(r2.E, abs=1e-13)
    assert np.abs(r1.gammas[perm] - r2.gammas).max() < 1e-12


# ------------------------------------------------------- whole-loop checks

def test_tiny_system_reaches_exact_ground_state():
    N, terms = si.anderson_terms(1, 1.3, 0.7)
    ham = si.anderson(1, 1.3, 0.7)
    e_ed = ed.even_sector_ground_energy(N, terms)
    _, es = sgs.run(ham, si.random_states(N, 3, seed=5), 0.05, 300)
    assert np.all(np.diff(es) <= 1e-12)
    assert es[-1] == pytest.approx(e_ed, abs=1e-10)


def test_free_fermion_closed_form():
    # U = 0, R = 1: E -> -Tr sqrt(A^T A) + e0, Gamma -> polar(A) (even parity here)
    ham = si.anderson(3, 0.0, 0.5)
    s = np.linalg.svd(ham.A, compute_uv=False)
    e_exact = -s.sum() + ham.e0
    polarA = sgs.purify(ham.A)
    assert pfaffian(polarA) == pytest.approx(1.0)
    g, es = sgs.run(ham, si.random_states(ham.N, 1, seed=0), 0.1, 400)
    assert es[-1] == pytest.approx(e_exact, abs=1e-9)
    assert np.abs(g[0] - polarA).max() < 1e-6


def test_variational_bound_and_monotone_descent_c1_size():
    # N = 16 modes (L = 7): E_k >= E_ED(even) and non-increasing
    N, terms = si.anderson_terms(7, 1.0, 0.5)
    ham = si.anderson(7, 1.0, 0.5)
    e_ed = ed.even_sector_ground_energy(N, terms)
    _, es = sgs.run(ham, si.random_states(N, 4, seed=0), 0.05, 8)
    assert np.all(es >= e_ed - 1e-12)
    assert np.all(np.diff(es) <= 1e-12)


# ------------------------------------------------------------- observables

def test_observables_match_bruteforce(tiny):
    ham, g, vecs = tiny
    N = ham.N
    E, lam, tab = sgs.energy(ham, g)
    psi = np.stack(vecs, 1) @ lam
    poly = si.spin_dot_poly((0, 1), (2, 3))
    ref = np.vdot(psi, fock.majorana_poly_operator(N, poly) @ psi)
    assert abs(ob.expectation(g, lam, tab.G, poly) - ref) < 1e-13
    for NA in (1, 2, 3):
        rho = np.outer(psi, psi.conj()).reshape(2 ** NA, 2 ** (N - NA), 2 ** NA, 2 ** (N - NA))
        rA = np.einsum("ajbj->ab", rho)
        assert ob.renyi2(g, lam, tab.G, 2 * NA) == pytest.approx(-math.log(np.trace(rA @ rA).real), abs=1e-12)


def test_integrated_correlation_sum_rule_for_singlet():
    # Sigma(L-1) = 0 when the total spin vanishes: check on the exact singlet
    N, terms = si.anderson_terms(1, 1.3, 0.7)
    ham = si.anderson(1, 1.3, 0.7)
    g, _ = sgs.run(ham, si.random_states(N, 3, seed=5), 0.05, 300)
    E, lam, tab = sgs.energy(ham, g)
    C = np.array([ob.expectation(g, lam, tab.G, si.spin_dot_poly((0, 1), (2 * r, 2 * r + 1))).real
                  for r in range(2)])
    assert ob.integrated_correlation(C)[-1] == pytest.approx(0.0, abs=1e-9)


# ---------------------------------------------------------------- exp-map update (App. A)

def test_exp_update_is_orthogonal_and_first_order_euler():
    """Eq. ExpStep: R Gamma R^T keeps Gamma pure to rounding; with the 1/4
    reading its first-order term is the Euler step of Eq. RKstep (the
    difference to polar(Gamma + ds dGamma) shrinks as ds^3), and the printed
    1/2 moves twice as far."""
    ham = si.anderson(2, 1.3, 0.6)
    g = si.random_states(ham.N, 3, seed=5)
    r = sgs.step(ham, g, 0.05)
    dg = r.dgamma
    for m in range(3):
        assert np.abs(dg[m] @ g[m] + g[m] @ dg[m]).max() < 1e-12  # tangent
        out = sgs.exp_update(g[m], dg[m], 0.05)
        assert np.abs(out @ out + np.eye(g.shape[1])).max() < 1e-13
        errs = []
        for ds in (0.02, 0.01, 0.005):
            e = np.abs(sgs.exp_update(g[m], dg[m], ds) - sgs.purify(g[m] + ds * dg[m])).max()
            errs.append(e)
        # both are second-order retractions: the generator anticommutes with
        # Gamma, so R Gamma R^T is the geodesic, and the polar projection
        # matches the geodesic through second order; the gap is O(ds^3)
        assert 6.5 < errs[0] / errs[1] < 9.5 and 6.5 < errs[1] / errs[2] < 9.5
        # first order: (exp_update - Gamma) / ds -> dGamma; the printed 1/2 -> 2 dGamma
        ds = 1e-5
        d1 = (sgs.exp_update(g[m], dg[m], ds) - g[m]) / ds
        d2 = (sgs.exp_update(g[m], dg[m], ds, coef=0.5) - g[m]) / ds
        scale = np.abs(dg[m]).max()
        assert np.abs(d1 - dg[m]).max() < 1e-3 * scale
        assert np.abs(d2 - 2 * dg[m]).max() < 1e-3 * scale


def test_exp_update_descends_and_reaches_ground_state():
    """N = 4, R = 3 with the exponential map: monotone descent to the exact
    even-sector ground state, as with the Euler step."""
    N, terms = si.anderson_terms(1, 1.3, 0.7)
    ham = si.anderson(1, 1.3, 0.7)
    e_ed = ed.even_sector_ground_energy(N, terms)
    _, es = sgs.run(ham, si.random_states(N, 3, seed=5), 0.05, 300, update="exp")
    assert np.all(np.diff(es) <= 1e-12)
    assert es[-1] == pytest.approx(e_ed, abs=1e-10)


# ---------------------------------------------------------------- variance

def _bruteforce_moments(ham, g, lam):
    """<H>, <H^2> of sum_mu lambda_mu |phi_mu> built in Fock space (same gauge as G)."""
    vecs = fock.fix_gauge([fock.gaussian_state(x) for x in g], fock.gaussian_state(g[0]))
    vecs = fock.fix_gauge(vecs, vecs[0])
    psi = np.stack(vecs, 1) @ lam
    H = fock.majorana_poly_operator(ham.N, ham.poly())
    nr = np.vdot(psi, psi).real
    hp = H @ psi
    return np.vdot(psi, hp).real / nr, np.vdot(hp, hp).real / nr


@pytest.mark.parametrize("model,R", [("anderson", 1), ("anderson", 3), ("tck", 2), ("tck", 3)])
def test_variance_definition_matches_bruteforce(model, R):
    """Eq. (residual): delta_H^2 = <H^2> - <H>^2 from H^2 multiplied out as
    Majorana words equals the Fock-space value (Anderson N = 4, two-channel
    Kondo N = 6, random states)."""
    ham = si.anderson(1, 1.3, 0.7) if model == "anderson" else si.two_channel_kondo(1, 0.9, U=2.0)
    g = si.random_states(ham.N, R, seed=5 + R)
    E, lam, tab = sgs.energy(ham, g)
    e1, e2, var = ob.hamiltonian_variance(ham, g, lam, tab.G)
    b1, b2 = _bruteforce_moments(ham, g, lam)
    assert abs(e1 - E) < 1e-12 * max(1.0, abs(E))
    assert abs(e1 - b1) < 1e-12 * max(1.0, abs(b1))
    assert abs(e2 - b2) < 1e-12 * max(1.0, abs(b2))
    assert abs(var - (b2 - b1 * b1)) < 1e-11 * max(1.0, b2)
    assert var > 0.0


@pytest.mark.parametrize("model", ["anderson", "tck"])
def test_variance_trace_form_matches_definition(model):
    """The matrix form (K = 1 + i Delta, <H2 H2>_t = <H2>_t^2 + Tr(alpha K
    alpha K^T) / 2, Pfaffians of 6 and 8 Majoranas for the quartic words)
    against the word expansion, n = 16 and 12, R = 3."""
    ham = si.anderson(3, 1.3, 0.7) if model == "anderson" else si.two_channel_kondo(1, 0.9, U=2.0)
    g = si.random_states(ham.N, 3, seed=2)
    E, lam, tab = sgs.energy(ham, g)
    a = ob.hamiltonian_variance(ham, g, lam, tab.G)
    b = ob.hamiltonian_variance_trace(ham, g, lam, tab.G)
    assert abs(a[0] - b[0]) < 1e-12 * max(1.0, abs(a[0]))
    assert abs(a[1] - b[1]) < 1e-12 * max(1.0, abs(a[1]))
    assert abs(a[2] - b[2]) < 1e-11 * max(1.0, a[1])


def test_variance_vanishes_on_an_eigenstate():
    """A quadratic H (U = 0) has the Gaussian ground state Gamma = -i sign(iA):
    delta_H^2 = 0 there (both forms), and > 0 on a random state."""
    ham = si.anderson(3, 0.0, 0.7)
    assert ham.quartic_idx.shape[0] == 0 or np.all(ham.quartic_val == 0.0)
    w, v = np.linalg.eigh(1j * ham.A)
    gam = (-1j * (v * np.sign(w)) @ v.conj().T).real
    gam = 0.5 * (gam - gam.T)
    assert np.abs(gam @ gam + np.eye(ham.n)).max() < 1e-12
    g = gam[None]
    lam = np.array([1.0 + 0.0j])
    G = np.ones((1, 1), dtype=complex)
    e1, e2, var = ob.hamiltonian_variance(ham, g, lam, G)
    t1, t2, tvar = ob.hamiltonian_variance_trace(ham, g, lam, G)
    assert abs(var) < 1e-12 * e2 and abs(tvar) < 1e-12 * t2
    assert abs(e1 - (ham.e0 - 0.5 * np.abs(2 * w).sum())) < 1e-12 * max(1.0, abs(e1))
    rnd = si.random_states(ham.N, 1, seed=4)
    assert ob.hamiltonian_variance(ham, rnd, lam, G)[2] > 1e-3


# ------------------------------------------------------------ rank growing

def test_small_rotations_are_special_orthogonal_near_one():
    for Q in si.small_rotations(12, 3, 0.3, seed=1):
        assert np.abs(Q @ Q.T - np.eye(12)).max() < 1e-14
        assert abs(np.linalg.det(Q) - 1.0) < 1e-13
        assert 0.25 < np.linalg.norm(Q - np.eye(12)) < 0.31


def test_grow_reaches_the_exact_ground_state():
    """Sec. III.C: from one random state (converging to GHF), rank 1 -> 3 by
    rotated copies of the largest-amplitude state; N = 4 Anderson reaches the
    exact even-sector ground energy, and never goes below it."""
    N, terms = si.anderson_terms(1, 1.3, 0.7)
    ham = si.MajoranaHamiltonian.from_poly(N, si.fermion_terms_to_majorana(terms))
    g0 = si.random_states(ham.N, 1, seed=3)[0]
    g, es, ranks = sgs.grow(ham, g0, 0.05, 40, si.small_rotations(ham.n, 2, 0.3, seed=1), mode="unit")
    ex = ed.even_sector_ground_energy(N, terms)
    assert g.shape[0] == 3 and ranks == [1] * 40 + [2] * 40 + [3] * 40
    assert abs(es[-1] - ex) < 1e-6
    assert es.min() > ex - 1e-10


def test_grow_additions_lower_the_energy():
    """N = 6: every added state lowers the energy at once (the variational
    space grows), the trajectory decreases, and stays above the exact value."""
    N, terms = si.anderson_terms(2, 1.3, 0.7)
    ham = si.MajoranaHamiltonian.from_poly(N, si.fermion_terms_to_majorana(terms))
    g0 = si.random_states(ham.N, 1, seed=3)[0]
    g, es, ranks = sgs.grow(ham, g0, 0.05, 40, si.small_rotations(ham.n, 2, 0.3, seed=1), mode="unit")
    assert np.all(np.diff(es) <= 1e-12)
    for r in (1, 2):
        assert es[40 * r] < es[40 * r - 1]
    assert es[-1] > ed.even_sector_ground_energy(N, terms)


def test_wilson_tail_hoppings_enter_the_chain():
    """Fig. 4 caption: L_W = 20 extra sites with t_n = Lambda^-n t, Lambda = 1.2.
    The last bath bond of the tail couples the last two sites with t_20."""
    tail = si.wilson_hoppings(20, 1.2)
    assert len(tail) == 20 and abs(tail[0] - 1 / 1.2) < 1e-15 and abs(tail[-1] - 1.2 ** -20) < 1e-15
    N, terms = si.anderson_terms(3, 1.0, 0.5, wilson_tail=tail)
    assert N == 2 * (1 + 3 + 20)
    hops = {}
    for c, ops in terms:
        if len(ops) == 2 and ops[0][1] and not ops[1][1] and ops[0][0] != ops[1][0]:
            hops[(ops[0][0], ops[1][0])] = c
    assert abs(hops[(si.siam_mode(22, 0), si.siam_mode(23, 0))] + 1.2 ** -20) < 1e-15


def test_renyi2_tensor_symmetries_and_split_form():
    """The terms of Eq. (S2_SGS) satisfy T(p, q) = T(q, p) and
    T(p*, q*) = T(p, q)^* with (a, b)* = (b, a), and the block Pfaffian of
    Eq. (pfMA) equals the split product Pf(K_q) Pf(K_p - K_q^{-1}) of
    Eq. (TrArho2_final) with either block inverted (App. B); summing w Re T
    over one representative per orbit reproduces S_2."""
    from oracle import gaussian as ga
    from oracle.pfaffian import pfaffian_log
    ham = si.anderson(5, 1.0, 0.5)
    R, nA = 3, 8
    g = si.random_states(ham.N, R, seed=3)
    E, lam, tab = sgs.energy(ham, g)
    K = {(a, b): (g[a] if a == b else ga.delta(g[a], g[b]))[:nA, :nA] for a in range(R) for b in range(R)}
    one = np.eye(nA)

    def pf(m):
        la, ph = pfaffian_log(m)
        return ph * math.exp(la)

    def term(a, b, c, d):
        coef = lam[a] * np.conj(lam[b]) * lam[c] * np.conj(lam[d]) * tab.G[b, a] * tab.G[d, c]
        return coef * pf(np.block([[K[a, b], 1j * one], [-1j * one, K[c, d]]])) / 2 ** (nA // 2)

    total = 0.0
    for p in range(R * R):
        for q in range(R * R):
            a, b = divmod(p, R)
            c, d = divmod(q, R)
            t = term(a, b, c, d)
            assert abs(t - term(c, d, a, b)) < 1e-12 * max(1.0, abs(t))
            assert abs(t - np.conj(term(b, a, d, c))) < 1e-12 * max(1.0, abs(t))
            z = pf(np.block([[K[a, b], 1j * one], [-1j * one, K[c, d]]]))
            for x, y in (((a, b), (c, d)), ((c, d), (a, b))):
                split = pf(K[y]) * pf(K[x] - np.linalg.inv(K[y]))
                assert abs(split - z) < 1e-10 * max(1.0, abs(z))
            # one representative per orbit, with the orbit's size
            cp, cq = sorted(((b * R + a), (d * R + c)))
            if p <= q and (cp, cq) >= (p, q):
                total += (1 if p == q else 2) * (1 if (cp, cq) == (p, q) else 2) * t.real
    assert -math.log(total) == pytest.approx(ob.renyi2(g, lam, tab.G, nA), abs=1e-12)


# ------------------------------------------------- interaction words, m > 4

def test_word_fock_reproduces_quartic_fock():
    """The cofactor form of the transition Fock matrix, applied to quartic
    words, is the paper's 6 U Delta (Sec. II.C)."""
    from oracle import gaussian as ga
    ham = si.anderson(2, 1.3, 0.6)
    g = si.random_states(ham.N, 2, seed=5)
    d = ga.delta(g[0], g[1])
    ref = ga.fock_matrix(ham, d) - ham.A
    got = sum(ga.word_fock(d, w, u) for w, u in zip(ham.quartic_idx, ham.quartic_val))
    assert np.abs(got - ref).max() < 1e-14


@pytest.mark.parametrize("mode", ["printed", "unit"])
@pytest.mark.parametrize("W3,W4", [(0.7, 0.0), (0.0, 0.5), (0.6, -0.4)])
def test_force_with_higher_words_matches_bruteforce(mode, W3, W4):
    """Words of 6 and 8 Majoranas (three- and four-body densities): the
    oracle's compact force (Eq. EOM-Gamma3 with the cofactor Fock matrix)
    against the Fock-space derivative of Eq. (EOM-Gamma2), and the pair
    tables against the projected Hamiltonian."""
    ham = si.anderson_multibody(1, 1.1, 0.6, W3, W4)
    assert len(ham.higher_idx) > 0
    g = si.random_states(ham.N, 3, seed=8)
    tab = sgs.pair_tables(ham, g)
    vecs = fock.fix_gauge([fock.gaussian_state(x) for x in g], fock.gaussian_state(g[0]))
    vecs = fock.fix_gauge(vecs, vecs[0])
    V = np.stack(vecs, 1)
    H = fock.majorana_poly_operator(ham.N, ham.poly())
    N, terms = si.anderson_multibody_terms(1, 1.1, 0.6, W3, W4)
    assert np.abs(H - fock.fermion_operator(N, terms)).max() < 1e-12
    assert np.abs(tab.h - V.conj().T @ H @ V).max() < 1e-12
    E, lam = sgs.solve_amplitudes(tab.G, tab.h)
    dg = sgs.forces(ham, g, tab, E, lam, mode)
    ref = _bruteforce_force(ham, g, mode)
    assert np.abs(dg - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())


def test_multibody_energy_descends_to_ed():
    """Imaginary-time steps with 6- and 8-Majorana words stay above the
    even-sector ground energy and descend (Sec. III.C)."""
    N, terms = si.anderson_multibody_terms(2, 1.0, 0.5, 0.8, -0.6)
    ham = si.anderson_multibody(2, 1.0, 0.5, 0.8, -0.6)
    e_ed = ed.even_sector_ground_energy(N, terms)
    _, es = sgs.run(ham, si.random_states(N, 3, seed=2), 0.05, 40)
    assert np.all(es >= e_ed - 1e-12)
    assert np.all(np.diff(es) <= 1e-12)
