"""Observables of an SGS state.

* Expectation of a Majorana polynomial O (Sec. IV.B uses the spin correlation
  C(r) = <S(0).S(r)>, Eq. (Cr)):
  <psi|O|psi> = sum_{mu,b} lambda_mu^* lambda_b G_{mu b} <O>_t(Delta^{b mu}),
  where <O>_t is the transition value from Wick's theorem (Sec. III.B).
* Integrated correlation, Eq. (integrated_correlation): Sigma(x) = 1 + sum_{r<=x} C(r)/C(0).
* Renyi-2 entropy of the first 2 N_A Majoranas, Eq. (S2_SGS):
  Tr rho_A^2 = sum_{a,b,g,d} lambda_a lambda_b^* lambda_g lambda_d^* G_ba G_dg
               Tr_A[ rho^{ab}_A rho^{gd}_A ],
  where rho^{ab} = |a><b| / <b|a> is a Gaussian operator whose restriction to A
  has two-point matrix Delta^{ab}_A (Delta^{aa} = Gamma^a), and for two such
  operators Tr(rho_1 rho_2) = 2^(-N_A) Pf([[D_1, i 1], [-i 1, D_2]]).
  This closed form replaces the coherent-state prefactors of App. B
  (Eqs. TrArho2_final, pfMA), which are hard to read in the source; it is
  pinned against brute-force reduced density matrices.
"""

from __future__ import annotations

import math

import numpy as np

from .gaussian import delta, poly_value
from .pfaffian import pfaffian_log


def expectation(gammas: np.ndarray, lam: np.ndarray, G: np.ndarray, poly) -> complex:
    R = gammas.shape[0]
    tot = 0.0
    for mu in range(R):
        for b in range(R):
            d = gammas[mu] if mu == b else delta(gammas[b], gammas[mu])  # Delta^{b mu}
            tot += np.conj(lam[mu]) * lam[b] * G[mu, b] * poly_value(d, poly)
    return tot


def integrated_correlation(C: np.ndarray) -> np.ndarray:
    """Sigma(x) for x = 0..len(C)-1, C[0] = C(0)."""
    return 1.0 + np.concatenate([[0.0], np.cumsum(C[1:] / C[0])])


def renyi2(gammas: np.ndarray, lam: np.ndarray, G: np.ndarray, nA: int) -> float:
    """S_2 = -ln Tr rho_A^2 for A = Majoranas 0..nA-1 (nA even)."""
    R = gammas.shape[0]
    NA = nA // 2
    D = {}
    for a in range(R):
        for b in range(R):
            D[a, b] = (gammas[a] if a == b else delta(gammas[a], gammas[b]))[:nA, :nA]
    I = np.eye(nA)
    tot = 0.0
    for a in range(R):
        for b in range(R):
            for g in range(R):
                for d in range(R):
                    coef = lam[a] * np.conj(lam[b]) * lam[g] * np.conj(lam[d]) * G[b, a] * G[d, g]
                    Z = np.block([[D[a, b], 1j * I], [-1j * I, D[g, d]]])
                    la, ph = pfaffian_log(Z)
                    tot += coef * ph * math.exp(la - NA * math.log(2.0))
    return float(-math.log(tot.real))
