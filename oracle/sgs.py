"""One imaginary-time step of the SGS method, written out from the paper.

Steps, in the paper's order (Sec. III.C: alternate the amplitude solve and the
covariance-matrix step):

1. Gram matrix G and projected Hamiltonian h (Sec. II.C):
   G_ab = <phi_a|phi_b>, h_ab = <phi_a|H|phi_b> = G_ab * <H>_t(Delta^{ba}).
2. Amplitudes from h lambda = E G lambda, Eq. (eigLambda), lowest E,
   normalized lambda^dag G lambda = 1; renormalized amplitudes
   lambda~_mu = <phi_mu|psi> = (G lambda)_mu (Sec. III.A).
3. Covariance-matrix force, Eq. (EOM-Gamma3), read with lambda~_mu^* as in
   Eq. (EOM-Gamma2) (the printed lambda~_mu in Eq. (EOM-Gamma3) drops the star):
   dG_mu = sum_b lambda_b lambda~_mu^* c_mu [ 2i G_mb [D, F] + 2 G_mb (D F D + F)
           - h_mb D + sum_g G_mg (G^-1 h)_gb Delta^{g mu} ] + c.c.,
   with D = Delta^{b mu}, F = F^{b mu};
   c_mu = 1 / (lambda_mu lambda~_mu^*) (printed choice, Sec. III.A) or the
   unit-modulus choice lambda~_mu lambda_mu^* / |lambda~_mu lambda_mu|.
4. First-order step, Eq. (RKstep), Gamma + ds dGamma, then the canonical form
   Eq. (CM-normal-form) with every lambda_j rescaled to unit modulus, i.e. the
   polar factor of the updated matrix (computed exactly with eigh).
   Alternative (App. A, Eq. ExpStep): the orthogonal update R Gamma R^T with
   R the matrix exponential of a multiple of [Gamma, dGamma] (scipy's expm),
   with the coefficient read so that its first-order term is the Euler step.

Rank growing (Sec. III.C, ``grow``): from one state, run steps, then add a
random special orthogonal transformation (close to 1) of the state of
largest amplitude, and repeat.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import scipy.linalg
import scipy.sparse as sparse

from .gaussian import delta, fock_matrix, overlap_table, poly_value, quartic_tensor


@dataclass
class PairTables:
    G: np.ndarray          # (R, R) complex Gram matrix
    h: np.ndarray          # (R, R) complex <phi_a|H|phi_b>
    logabs: np.ndarray     # log|G|
    arg: np.ndarray        # arg G
    eps: np.ndarray        # h_ab / G_ab


def pair_tables(ham, gammas: np.ndarray, use_direct: bool = False, hpoly=None) -> PairTables:
    R = gammas.shape[0]
    la, ar = overlap_table(gammas, use_direct)
    G = np.exp(la) * np.exp(1j * ar)
    hp = ham.poly() if hpoly is None else hpoly
    eps = np.zeros((R, R), dtype=complex)
    for a in range(R):
        for b in range(R):
            d = gammas[a] if a == b else delta(gammas[b], gammas[a])  # Delta^{ba}
            eps[a, b] = poly_value(d, hp)
    h = G * eps
    return PairTables(G=G, h=h, logabs=la, arg=ar, eps=eps)


def canonical_basis(G: np.ndarray, rel_threshold: float = 1e-12) -> np.ndarray:
    """X = U_kept diag(s_kept)^(-1/2) of canonical orthogonalization: the
    eigenvectors of (the Hermitian part of) G whose eigenvalue exceeds
    rel_threshold * the largest; X^dag G X = 1, and X X^dag is the inverse of G
    on the kept subspace (G^-1 itself when nothing is dropped)."""
    Gh = 0.5 * (G + G.conj().T)
    s, U = np.linalg.eigh(Gh)
    keep = s > rel_threshold * s.max()
    return U[:, keep] / np.sqrt(s[keep])[None, :]


def solve_amplitudes(G: np.ndarray, h: np.ndarray, rel_threshold: float = 1e-12):
    """Lowest (E, lambda) of h lambda = E G lambda after canonical orthogonalization
    (eigenvectors of G below rel_threshold * max eigenvalue are dropped)."""
    hh = 0.5 * (h + h.conj().T)
    X = canonical_basis(G, rel_threshold)
    hp = X.conj().T @ hh @ X
    e, y = np.linalg.eigh(0.5 * (hp + hp.conj().T))
    lam = X @ y[:, 0]
    return float(e[0]), lam


# Vanishing amplitudes (Sec. III.A notes that the printed choice diverges as
# some lambda_mu -> 0; the paper fixes no rule).  Readings used here and by
# the GPU path:
#  * printed: the force on mu carries lambda_b / lambda_mu (exactly 1 for
#    b = mu).  When |lambda_mu| <= LAMBDA_FLOOR max|lambda|, lambda_mu is at
#    the rounding floor of any float64 eigen-solver (LAPACK's tridiagonal
#    solvers return exact zeros there), the ratio carries no information, and
#    the state is left unchanged by the step (its weight is 0).
#  * unit: w_mu lambda_b = |lambda~_mu| (lambda_mu^* / |lambda_mu|) lambda_b with
#    the phase lambda_mu^* / |lambda_mu| read as 1 when lambda_mu = 0.
LAMBDA_FLOOR = 1e-13


def weights(lam: np.ndarray, lamt: np.ndarray, mode: str = "printed") -> np.ndarray:
    """c_mu of Eq. (Bmu): printed 1 / (lambda_mu lambda~_mu^*), or the
    unit-modulus lambda~_mu lambda_mu^* / |lambda~_mu lambda_mu| (phase of a
    vanishing product read as the phase of lambda~_mu, i.e. lambda_mu's as 1)."""
    if mode == "printed":
        with np.errstate(divide="ignore", invalid="ignore"):
            return 1.0 / (lam * lamt.conj())
    if mode == "unit":
        ph_lam = np.ones(lam.shape, dtype=complex)
        nz = np.abs(lam) > 0
        ph_lam[nz] = lam[nz].conj() / np.abs(lam[nz])
        ph_lt = np.ones(lam.shape, dtype=complex)
        nzt = np.abs(lamt) > 0
        ph_lt[nzt] = lamt[nzt] / np.abs(lamt[nzt])
        return ph_lt * ph_lam
    raise ValueError(mode)


def term_weights(lam: np.ndarray, lamt: np.ndarray, mode: str = "printed") -> np.ndarray:
    """K[mu, b] = c_mu lambda~_mu^* lambda_b, the factor of the (mu, b) term of
    Eq. (EOM-Gamma3), with the readings for vanishing amplitudes above."""
    R = lam.shape[0]
    if mode == "printed":
        K = np.zeros((R, R), dtype=complex)
        lmax = np.abs(lam).max()
        for mu in range(R):
            if np.abs(lam[mu]) > LAMBDA_FLOOR * lmax:
                K[mu] = lam / lam[mu]
                K[mu, mu] = 1.0
        return K
    c = weights(lam, lamt, mode)
    return (c * lamt.conj())[:, None] * lam[None, :]


def forces(ham, gammas: np.ndarray, tab: PairTables, E: float, lam: np.ndarray,
           mode: str = "printed", rel_threshold: float = 1e-12) -> np.ndarray:
    """dGamma_mu / ds for every state, Eq. (EOM-Gamma3) in its printed long form.

    G^-1 in the projector of Eq. (projImEvol) is read, like the amplitude
    solve, through canonical orthogonalization: X X^dag, the inverse of G on
    the kept subspace (G^-1 when nothing is dropped).  Then V X X^dag V^dag is
    the orthogonal projector onto the span of the kept combinations of states."""
    R, n, _ = gammas.shape
    G, h = tab.G, tab.h
    lamt = G @ lam
    Kw = term_weights(lam, lamt, mode)
    X = canonical_basis(G, rel_threshold)
    Ginv_h = X @ (X.conj().T @ h)
    qt = quartic_tensor(ham)
    out = np.zeros((R, n, n))
    for mu in range(R):
        D = np.stack([gammas[mu] if b == mu else delta(gammas[b], gammas[mu])
                      for b in range(R)])  # Delta^{b mu}
        # sum_g G_{mu g} (G^-1 h)_{g b} Delta^{g mu} for every b at once
        K = G[mu][:, None] * Ginv_h  # K[g, b]
        norm_terms = np.tensordot(K.T, D, axes=(1, 0))
        acc = np.zeros((n, n), dtype=complex)
        for b in range(R):
            F = sparse.csr_matrix(fock_matrix(ham, D[b], qt))
            DF = (F.T @ D[b].T).T   # D F (F sparse)
            FD = F @ D[b]
            term = (2j * G[mu, b] * (DF - FD)
                    + 2.0 * G[mu, b] * (DF @ D[b] + F.toarray())
                    - h[mu, b] * D[b]
                    + norm_terms[b])
            acc += Kw[mu, b] * term
        out[mu] = (acc + acc.conj()).real
    return out


def purify(x: np.ndarray) -> np.ndarray:
    """Polar factor of a real skew matrix: canonical form with unit lambda_j."""
    x = 0.5 * (x - x.T)
    s, V = np.linalg.eigh(1j * x)  # i x is Hermitian
    g = (-1j * (V * np.sign(s)[None, :]) @ V.conj().T).real
    return 0.5 * (g - g.T)


# Exponential-map update (App. A, Eq. ExpStep): Gamma <- R Gamma R^T with R
# the exponential of a multiple of the commutator [Gamma, dGamma].  For a
# tangent dGamma (it anticommutes with Gamma, pinned) [[Gamma, dGamma], Gamma]
# = 4 dGamma, so R = exp(c ds [Gamma, dGamma]) moves Gamma by 2 c ds dGamma to
# first order: c = 1/4 agrees with the Euler step of Eq. RKstep, the printed
# c = 1/2 takes a step of 2 ds.  EXP_COEF is the reading used here.
EXP_COEF = 0.25


def exp_update(g: np.ndarray, dg: np.ndarray, dtau: float, coef: float = EXP_COEF) -> np.ndarray:
    K = coef * dtau * (g @ dg - dg @ g)
    K = 0.5 * (K - K.T)
    Rm = scipy.linalg.expm(K)
    out = Rm @ g @ Rm.T
    return 0.5 * (out - out.T)


@dataclass
class StepResult:
    gammas: np.ndarray
    E: float
    lam: np.ndarray
    tables: PairTables
    dgamma: np.ndarray


def step(ham, gammas: np.ndarray, dtau: float, mode: str = "printed",
         rel_threshold: float = 1e-12, hpoly=None, update: str = "euler") -> StepResult:
    """One step: tables, amplitudes, force, then either the Euler step with
    purification (Eqs. RKstep, CM-normal-form) or the exponential map
    (Eq. ExpStep), update = "euler" | "exp"."""
    tab = pair_tables(ham, gammas, hpoly=hpoly)
    E, lam = solve_amplitudes(tab.G, tab.h, rel_threshold)
    dg = forces(ham, gammas, tab, E, lam, mode, rel_threshold)
    if update == "exp":
        new = np.stack([exp_update(gammas[m], dg[m], dtau) for m in range(gammas.shape[0])])
    else:
        new = np.stack([purify(gammas[m] + dtau * dg[m]) for m in range(gammas.shape[0])])
    return StepResult(gammas=new, E=E, lam=lam, tables=tab, dgamma=dg)


def energy(ham, gammas: np.ndarray, hpoly=None):
    tab = pair_tables(ham, gammas, hpoly=hpoly)
    E, lam = solve_amplitudes(tab.G, tab.h)
    return E, lam, tab


def run(ham, gammas: np.ndarray, dtau: float, nsteps: int, mode: str = "printed",
        callback=None, update: str = "euler") -> tuple:
    """nsteps steps; returns (final gammas, energies of the states entering each step)."""
    hp = ham.poly()
    es: List[float] = []
    g = gammas
    for k in range(nsteps):
        r = step(ham, g, dtau, mode, hpoly=hp, update=update)
        es.append(r.E)
        g = r.gammas
        if callback is not None:
            callback(k, r)
    return g, np.array(es)


def grow(ham, gamma0: np.ndarray, dtau: float, steps_per_rank: int, rotations, mode: str = "printed",
         update: str = "euler") -> tuple:
    """Rank-growing protocol of Sec. III.C: steps_per_rank steps from the
    starting state(s); then, per rotation Q, add Q Gamma_a Q^T for the state a
    of largest |lambda_a| and run steps_per_rank more steps.  Returns
    (final gammas, energies of the states entering every step, rank of every
    step)."""
    g = gamma0[None] if gamma0.ndim == 2 else gamma0
    es: List[float] = []
    ranks: List[int] = []
    for r in range(len(rotations) + 1):
        g, e = run(ham, g, dtau, steps_per_rank, mode, update=update)
        es.extend(e)
        ranks.extend([g.shape[0]] * steps_per_rank)
        if r == len(rotations):
            break
        _, lam, _ = energy(ham, g)
        a = int(np.argmax(np.abs(lam)))
        new = rotations[r] @ g[a] @ rotations[r].T
        g = np.concatenate([g, (0.5 * (new - new.T))[None]])
    return g, np.array(es), ranks
