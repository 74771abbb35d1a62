"""Gaussian-state algebra in the covariance-matrix formalism (Sec. II.B, III.B).

* Overlap magnitude (cited to Bravyi & Gosset in Sec. II.B):
  |<a|b>|^2 = 2^(-N) |Pf(Gamma_a + Gamma_b)|, so
  log|<a|b>| = -(N/2) ln 2 + (1/4) ln|det(Gamma_a + Gamma_b)|.
* Phase in the reference gauge of Sec. II.B (<phi_0|phi_mu> real positive):
  the gauge-invariant triple product
  <r|a><a|b><b|r> = 4^(-N) i^N Pf([[i G_r, -1, 1], [1, i G_a, -1], [-1, 1, i G_b]])
  (Bravyi & Gosset), and its Schur-reduced form
  = 4^(-N) i^N Pf(i G_r) Pf(i (G_a + G_r)) Pf(C_ab),
  C_ab = i (G_b + G_r) - i (1 - i G_r)(G_a + G_r)^(-1)(1 + i G_r).
* Transition matrix, Eq. (def-delta-matrix):
  Delta^{ab} = [i (G_a - G_b) - 2] (G_a + G_b)^(-1), with
  <phi_b| c_k c_l |phi_a> = i G_ba Delta^{ab}_kl for k != l, and a product of
  m distinct sorted Majoranas has transition value i^(m/2) Pf(Delta^{ab}[w, w]).
* Generalized Fock matrix (Sec. III.B): F^{ab}_kl = A_kl + 6 sum_mn U_klmn Delta^{ab}_mn,
  with U the fully antisymmetric quartic tensor of Sec. II.A.
"""

from __future__ import annotations

import itertools
import math
from typing import Dict, Tuple

import numpy as np

from .pfaffian import pfaffian, pfaffian_log

LN2 = math.log(2.0)


def log_abs_overlap(ga: np.ndarray, gb: np.ndarray) -> float:
    N = ga.shape[0] // 2
    sign, logdet = np.linalg.slogdet(ga + gb)
    if sign == 0:
        return -math.inf
    return -0.5 * N * LN2 + 0.25 * logdet


def triple_product_direct(gr: np.ndarray, ga: np.ndarray, gb: np.ndarray) -> Tuple[float, complex]:
    """(log|T|, T/|T|) of T = <r|a><a|b><b|r> from the 3n x 3n Pfaffian."""
    n = gr.shape[0]
    N = n // 2
    I = np.eye(n)
    Z = np.block([[1j * gr, -I, I], [I, 1j * ga, -I], [-I, I, 1j * gb]])
    la, ph = pfaffian_log(Z)
    return la - N * 2 * LN2, ph * (1j ** (N % 4))


def schur_matrix(gr: np.ndarray, ga: np.ndarray, gb: np.ndarray) -> np.ndarray:
    n = gr.shape[0]
    I = np.eye(n)
    w = np.linalg.inv(ga + gr)
    return 1j * (gb + gr) - 1j * (I - 1j * gr) @ w @ (I + 1j * gr)


def triple_product_schur(gr: np.ndarray, ga: np.ndarray, gb: np.ndarray) -> Tuple[float, complex]:
    """Same triple product via Pf(i G_r) Pf(i (G_a + G_r)) Pf(C_ab)."""
    n = gr.shape[0]
    N = n // 2
    l1, p1 = pfaffian_log(1j * gr)
    l2, p2 = pfaffian_log(1j * (ga + gr))
    l3, p3 = pfaffian_log(schur_matrix(gr, ga, gb))
    return l1 + l2 + l3 - N * 2 * LN2, p1 * p2 * p3 * (1j ** (N % 4))


def overlap_table(gammas: np.ndarray, use_direct: bool = False) -> Tuple[np.ndarray, np.ndarray]:
    """(log|G|, arg G) for the Gram matrix G_ab = <phi_a|phi_b>, gauge <phi_0|phi_mu> > 0."""
    R, n, _ = gammas.shape
    N = n // 2
    logabs = np.zeros((R, R))
    arg = np.zeros((R, R))
    for a in range(R):
        for b in range(a + 1, R):
            logabs[a, b] = logabs[b, a] = log_abs_overlap(gammas[a], gammas[b])
    g0 = gammas[0]
    I = np.eye(n)
    if not use_direct:
        # factors of the Schur-reduced triple product that depend on (0, a) only
        _, p0 = pfaffian_log(1j * g0)
        pa = {}
        xa = {}
        for a in range(1, R):
            _, pa[a] = pfaffian_log(1j * (gammas[a] + g0))
            xa[a] = (I - 1j * g0) @ np.linalg.inv(gammas[a] + g0) @ (I + 1j * g0)
    for a in range(1, R):
        for b in range(a + 1, R):
            # <0|a><a|b><b|0> with <0|a>, <b|0> real positive: arg G_ab = arg T
            if use_direct:
                _, ph = triple_product_direct(g0, gammas[a], gammas[b])
            else:
                _, pc = pfaffian_log(1j * (gammas[b] + g0) - 1j * xa[a])
                ph = p0 * pa[a] * pc * (1j ** (N % 4))
            th = float(np.angle(ph))
            arg[a, b] = th
            arg[b, a] = -th
    return logabs, arg


def gram(gammas: np.ndarray, use_direct: bool = False) -> np.ndarray:
    la, ar = overlap_table(gammas, use_direct)
    return np.exp(la) * np.exp(1j * ar)


def delta(ga: np.ndarray, gb: np.ndarray) -> np.ndarray:
    """Delta^{ab} of Eq. (def-delta-matrix)."""
    n = ga.shape[0]
    return (1j * (ga - gb) - 2.0 * np.eye(n)) @ np.linalg.inv(ga + gb)


def word_value(d: np.ndarray, word) -> complex:
    """Transition value of the sorted distinct Majorana word: i^(m/2) Pf(Delta[w, w])."""
    m = len(word)
    if m == 0:
        return 1.0
    if m % 2:
        return 0.0
    idx = list(word)
    if m == 2:  # the Pfaffian of a 2x2 skew block is its upper entry
        return 1j * d[idx[0], idx[1]]
    return (1j ** (m // 2)) * pfaffian(d[np.ix_(idx, idx)].astype(complex))


def poly_value(d: np.ndarray, poly) -> complex:
    """Transition value <phi_b|O|phi_a> / G_ba for d = Delta^{ab} and O a Majorana polynomial."""
    return sum(coef * word_value(d, w) for w, coef in poly.items())


def quartic_tensor(ham) -> Tuple[np.ndarray, np.ndarray]:
    """(impurity Majorana list, dense antisymmetric U on it) with U = u/24 per ordering."""
    imp = ham.impurity_majoranas()
    pos = {int(k): i for i, k in enumerate(imp)}
    M = len(imp)
    U = np.zeros((M, M, M, M))
    for word, u in zip(ham.quartic_idx, ham.quartic_val):
        loc = [pos[int(k)] for k in word]
        for perm in itertools.permutations(range(4)):
            # sign of the permutation
            p = list(perm)
            s = 1
            for i in range(4):
                for j in range(i + 1, 4):
                    if p[i] > p[j]:
                        s = -s
            U[tuple(loc[x] for x in perm)] += s * u / 24.0
    return imp, U


def word_fock(d: np.ndarray, word, coef: complex) -> np.ndarray:
    """Transition Fock matrix of one word term coef * c_w0 ... c_w(m-1) (m even).

    F = A + 6 U Delta (Sec. II.C) is minus the derivative of the transition
    value <H>_t = e0 - sum_kl A_kl Delta_kl - sum_q u_q Pf(Delta[q]) with
    respect to the entries Delta_kl, k < l, halved (each enters twice in the
    quadratic part).  Read that way it extends to a word of any length, whose
    value is i^(m/2) Pf(Delta[w]) (Wick's theorem, Sec. III.B): for positions
    a < b of the word, with the Pfaffian cofactor of entry (a, b),
      F[w_a, w_b] = -(1/2) coef i^(m/2) (-1)^(a+b+1) Pf(Delta[w without a, b]),
    and F[w_b, w_a] = -F[w_a, w_b].  For quartic words this is 6 U Delta."""
    idx = list(word)
    m = len(idx)
    out = np.zeros(d.shape, dtype=complex)
    for a in range(m):
        for b in range(a + 1, m):
            rest = [idx[t] for t in range(m) if t != a and t != b]
            pf = pfaffian(d[np.ix_(rest, rest)].astype(complex)) if rest else 1.0
            v = -0.5 * coef * (1j ** (m // 2)) * (-1) ** (a + b + 1) * pf
            out[idx[a], idx[b]] += v
            out[idx[b], idx[a]] -= v
    return out


def fock_matrix(ham, d: np.ndarray, qt=None) -> np.ndarray:
    """F = A + 6 sum_mn U_klmn Delta_mn (complex in general), plus the
    contribution of every word of 6 or 8 Majoranas (word_fock)."""
    imp, U = quartic_tensor(ham) if qt is None else qt
    F = ham.A.astype(complex)
    if len(imp):
        blk = d[np.ix_(imp, imp)]
        F[np.ix_(imp, imp)] += 6.0 * np.einsum("klmn,mn->kl", U, blk)
    for w, v in zip(getattr(ham, "higher_idx", ()), getattr(ham, "higher_val", ())):
        F += word_fock(d, w, v * ham.word_phase(len(w)))
    return F
