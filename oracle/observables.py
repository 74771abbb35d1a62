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
* Variance of the Hamiltonian, Eq. (residual): delta_H^2 = <H^2> - <H>^2
  (Sec. IV.A).  ``hamiltonian_variance`` is the definition written out: H as
  a Majorana polynomial (H = e0 + i sum A_kl c_k c_l + sum_q u_q c c c c,
  Sec. II.A), H^2 multiplied out with c_k^2 = 1 and c_k c_l = -c_l c_k, every
  word evaluated by Wick's theorem (small systems only: H^2 has W^2 words).
  ``hamiltonian_variance_trace`` gives the same numbers for any size: on the
  transition operator of a pair, Wick's theorem holds for any product with
  the two-point matrix K = 1 + i Delta (K_kl = <c_k c_l>_t, K_kk = 1), so for
  H2 = sum_{k<l} alpha_kl c_k c_l (alpha = 2 i A)
    <H2>_t = (1/2) sum_kl alpha_kl K_kl,
    <H2 H2>_t = <H2>_t^2 + (1/2) Tr(alpha K alpha K^T),
  and a product with quartic words is the Pfaffian of the contraction matrix
  of its 6 or 8 Majoranas (M_ab = K_{i_a i_b}, a < b).  It is pinned against
  the definition.
"""

from __future__ import annotations

import itertools
import math
from typing import Dict, List, Tuple

import numpy as np
import scipy.sparse as sp

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


# ----------------------------------------------------------------- variance

def _word_product(w1, w2) -> Tuple[int, tuple]:
    """c_{w1} c_{w2} = sign * c_{w} with w sorted and distinct."""
    out: List[int] = []
    sign = 1
    for x in list(w1) + list(w2):
        out.append(x)
        i = len(out) - 1
        while i > 0 and out[i - 1] > out[i]:  # move c_x left: one anticommutation each
            out[i - 1], out[i] = out[i], out[i - 1]
            sign = -sign
            i -= 1
        if i > 0 and out[i - 1] == out[i]:    # c_x c_x = 1
            del out[i - 1:i + 1]
    return sign, tuple(out)


def hamiltonian_words(ham) -> Dict[tuple, complex]:
    """H = e0 + sum_{k<l} 2 i A_kl c_k c_l + sum_q u_q c_q0 c_q1 c_q2 c_q3 as sorted words."""
    h: Dict[tuple, complex] = {}
    if ham.e0:
        h[()] = complex(ham.e0)
    ks, ls = np.nonzero(np.triu(ham.A, 1))
    for k, l in zip(ks, ls):
        key = (int(k), int(l))
        h[key] = h.get(key, 0.0) + 2j * ham.A[k, l]
    for w, u in zip(ham.quartic_idx, ham.quartic_val):
        key = tuple(int(x) for x in w)
        h[key] = h.get(key, 0.0) + complex(u)
    return h


def square_words(h: Dict[tuple, complex]) -> Dict[tuple, complex]:
    out: Dict[tuple, complex] = {}
    for w1, c1 in h.items():
        for w2, c2 in h.items():
            s, w = _word_product(w1, w2)
            out[w] = out.get(w, 0.0) + s * c1 * c2
    return out


def hamiltonian_variance(ham, gammas: np.ndarray, lam: np.ndarray, G: np.ndarray):
    """(<H>, <H^2>, delta_H^2) of the SGS state, by the definition."""
    h = hamiltonian_words(ham)
    nrm = expectation(gammas, lam, G, {(): 1.0})
    e1 = expectation(gammas, lam, G, h) / nrm
    e2 = expectation(gammas, lam, G, square_words(h)) / nrm
    return float(e1.real), float(e2.real), float((e2 - e1 * e1).real)


def _matchings(m: int):
    """Perfect matchings of 0..m-1 with their signs (the terms of a Pfaffian)."""
    if m == 0:
        return [(1, [])]
    out = []
    for j in range(1, m):
        rest = [x for x in range(1, m) if x != j]
        for sg, pairs in _matchings(m - 2):
            out.append(((-1) ** (j - 1) * sg, [(0, j)] + [(rest[a], rest[b]) for a, b in pairs]))
    return out


_MATCH = {m: _matchings(m) for m in (4, 6, 8)}


def _pf_contraction(K: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """<c_i0 c_i1 ... > = Pf(M), M_ab = K[i_a, i_b] (a < b), for a batch of
    index rows idx (..., m)."""
    m = idx.shape[-1]
    tot = 0.0
    for sg, pairs in _MATCH[m]:
        t = sg
        for a, b in pairs:
            t = t * K[idx[..., a], idx[..., b]]
        tot = tot + t
    return tot


def hamiltonian_variance_trace(ham, gammas: np.ndarray, lam: np.ndarray, G: np.ndarray):
    """(<H>, <H^2>, delta_H^2) from the matrix form of Wick's theorem."""
    R = gammas.shape[0]
    n = ham.n
    alpha = 2j * ham.A
    asp = sp.csr_matrix(alpha)
    ks, ls = np.nonzero(np.triu(ham.A, 1))
    av = alpha[ks, ls]
    words = np.array(ham.quartic_idx, dtype=np.int64).reshape(-1, 4)
    us = np.array(ham.quartic_val, dtype=float)
    kl = np.stack([ks, ls], 1).astype(np.int64)
    s1 = s2 = nrm = 0.0
    for mu in range(R):
        for b in range(R):
            d = gammas[mu] if mu == b else delta(gammas[b], gammas[mu])  # Delta^{b mu}
            K = np.eye(n) + 1j * d
            h2 = 0.5 * np.sum(alpha * K)
            T = asp @ K
            S = asp @ K.T
            h2h2 = h2 * h2 + 0.5 * np.sum(T * S.T)
            h4 = h24 = h42 = h44 = 0.0
            for q in range(words.shape[0]):
                w = words[q]
                h4 += us[q] * _pf_contraction(K, w[None, :])[0]
                if len(av):
                    rows = np.concatenate([kl, np.repeat(w[None, :], len(av), 0)], 1)
                    h24 += us[q] * np.sum(av * _pf_contraction(K, rows))
                    rows = np.concatenate([np.repeat(w[None, :], len(av), 0), kl], 1)
                    h42 += us[q] * np.sum(av * _pf_contraction(K, rows))
                for q2 in range(words.shape[0]):
                    both = np.concatenate([w, words[q2]])[None, :]
                    h44 += us[q] * us[q2] * _pf_contraction(K, both)[0]
            c = np.conj(lam[mu]) * lam[b] * G[mu, b]
            s1 += c * (h2 + h4)
            s2 += c * (h2h2 + h24 + h42 + h44)
            nrm += c
    x, y = s1 / nrm, s2 / nrm
    e0 = ham.e0
    return float((e0 + x).real), float((e0 * e0 + 2 * e0 * x + y).real), float((y - x * x).real)
