"""Jordan-Wigner Fock-space operators for brute-force checks.

Mode j is tensor factor j (basis index x = sum_j n_j 2^(N-1-j));
a_j = Z x ... x Z x |0><1| x 1 x ... x 1, and the Majoranas follow
a_j = (c_2j + i c_2j+1)/2, i.e. c_2j = a_j + a_j^dag, c_2j+1 = -i (a_j - a_j^dag).

A Gaussian state with covariance matrix Gamma (Eq. CMdef) is the unique ground
state of (i/2) sum_kl Gamma_kl c_k c_l (energy -N).
"""

from __future__ import annotations

from functools import lru_cache
from typing import List, Sequence, Tuple

import numpy as np
import scipy.sparse as sp

_SM = np.array([[0.0, 1.0], [0.0, 0.0]])  # |0><1|
_Z = np.array([[1.0, 0.0], [0.0, -1.0]])
_I = np.eye(2)


def annihilators_sparse(N: int) -> List[sp.csr_matrix]:
    ops = []
    for j in range(N):
        m = sp.identity(1, format="csr")
        for k in range(N):
            f = _Z if k < j else (_SM if k == j else _I)
            m = sp.kron(m, sp.csr_matrix(f), format="csr")
        ops.append(m.tocsr())
    return ops


@lru_cache(maxsize=8)
def _annihilators_dense(N: int) -> Tuple[np.ndarray, ...]:
    return tuple(np.asarray(a.todense()) for a in annihilators_sparse(N))


def annihilators(N: int) -> List[np.ndarray]:
    return list(_annihilators_dense(N))


@lru_cache(maxsize=8)
def _majoranas(N: int) -> Tuple[np.ndarray, ...]:
    out = []
    for a in _annihilators_dense(N):
        ad = a.conj().T
        out.append((a + ad).astype(complex))
        out.append((-1j * (a - ad)).astype(complex))
    return tuple(out)


def majoranas(N: int) -> List[np.ndarray]:
    return list(_majoranas(N))


def fermion_operator(N: int, terms) -> np.ndarray:
    """Dense matrix of sum coef * prod ops built from a_j directly (no Majoranas)."""
    a = annihilators(N)
    dim = 2 ** N
    out = np.zeros((dim, dim), dtype=complex)
    for coef, ops in terms:
        m = np.eye(dim, dtype=complex) * coef
        for mode, dag in ops:
            m = m @ (a[mode].T if dag else a[mode])  # real matrices: dagger = transpose
        out += m
    return out


def fermion_operator_sparse(N: int, terms) -> sp.csr_matrix:
    a = annihilators_sparse(N)
    adag = [x.T.tocsr() for x in a]
    dim = 2 ** N
    out = sp.csr_matrix((dim, dim), dtype=complex)
    for coef, ops in terms:
        m = sp.identity(dim, format="csr", dtype=complex) * coef
        for mode, dag in ops:
            m = m @ (adag[mode] if dag else a[mode])
        out = out + m
    return out.tocsr()


def majorana_poly_operator(N: int, poly) -> np.ndarray:
    """Dense matrix of a Majorana polynomial {word: coef}."""
    c = majoranas(N)
    dim = 2 ** N
    out = np.zeros((dim, dim), dtype=complex)
    for word, coef in poly.items():
        m = np.eye(dim, dtype=complex) * coef
        for k in word:
            m = m @ c[k]
        out += m
    return out


def parity_operator(N: int) -> np.ndarray:
    dim = 2 ** N
    occ = np.array([bin(x).count("1") for x in range(dim)])
    return np.diag((-1.0) ** occ)


def gaussian_state(gamma: np.ndarray) -> np.ndarray:
    """Normalized ground vector of (i/2) sum Gamma_kl c_k c_l (arbitrary global phase)."""
    n = gamma.shape[0]
    N = n // 2
    c = majoranas(N)
    h = np.zeros((2 ** N, 2 ** N), dtype=complex)
    for k in range(n):
        for l in range(n):
            if gamma[k, l] != 0:
                h += 0.5j * gamma[k, l] * (c[k] @ c[l])
    w, v = np.linalg.eigh(h)
    if w[1] - w[0] < 1e-8:
        raise ValueError("covariance matrix is not pure: degenerate ground state")
    return v[:, 0]


def covariance(psi: np.ndarray, N: int) -> np.ndarray:
    """Gamma_kl = (-i/2) <[c_k, c_l]> of a normalized state (Eq. CMdef)."""
    c = majoranas(N)
    n = 2 * N
    g = np.zeros((n, n))
    for k in range(n):
        ck = c[k] @ psi
        for l in range(n):
            if k == l:
                continue
            cl = c[l] @ psi
            comm = np.vdot(psi, c[k] @ cl) - np.vdot(psi, c[l] @ ck)
            g[k, l] = float(np.real(-0.5j * comm))
    return g


def fix_gauge(states: Sequence[np.ndarray], ref: np.ndarray) -> List[np.ndarray]:
    """Multiply each vector by a phase so that <ref|phi> is real and positive."""
    out = []
    for s in states:
        ov = np.vdot(ref, s)
        out.append(s * (abs(ov) / ov) if abs(ov) > 0 else s)
    return out
