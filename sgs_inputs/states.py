"""Seeded initial covariance matrices.

Every initial Gaussian state is a Haar-random proper rotation applied to the
vacuum covariance matrix, ``Gamma = Q Gamma_0 Q^T`` with ``Q`` in SO(2N) drawn
by the QR recipe (sign-fixed so the distribution is Haar, then the first column
flipped when ``det Q < 0``).  Such states are pure and keep the vacuum's even
parity.
"""

from __future__ import annotations

import numpy as np


def vacuum_cm(N: int) -> np.ndarray:
    """Covariance matrix of the vacuum for a_j = (c_2j + i c_2j+1)/2."""
    g = np.zeros((2 * N, 2 * N))
    for j in range(N):
        g[2 * j, 2 * j + 1] = 1.0
        g[2 * j + 1, 2 * j] = -1.0
    return g


def haar_so(n: int, rng: np.random.Generator) -> np.ndarray:
    z = rng.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.slogdet(q)[0] < 0:
        q[:, 0] = -q[:, 0]
    return q


def random_states(N: int, R: int, seed: int = 0,
                  rng: np.random.Generator | None = None) -> np.ndarray:
    """(R, 2N, 2N) float64 stack of seeded Haar-random pure covariance matrices."""
    if rng is None:
        rng = np.random.default_rng(seed)
    g0 = vacuum_cm(N)
    n = 2 * N
    out = np.empty((R, n, n))
    for mu in range(R):
        q = haar_so(n, rng)
        g = q @ g0 @ q.T
        out[mu] = 0.5 * (g - g.T)
    return out


def small_rotations(n: int, count: int, eps: float, seed: int = 0) -> list:
    """count seeded special orthogonal n x n matrices Q = exp(eps K / |K|_F)
    with K a Gaussian random skew matrix, so |Q - 1|_F ~ eps: the
    transformations that create new states in the rank-growing protocol
    (Sec. III.C), passed to both the oracle and the GPU driver."""
    import scipy.linalg

    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        z = rng.standard_normal((n, n))
        k = z - z.T
        out.append(scipy.linalg.expm(eps * k / np.linalg.norm(k)))
    return out


def near_copy_states(N: int, R: int, eps: float, seed: int = 0) -> np.ndarray:
    """(R, 2N, 2N) chain of states, each a small seeded special orthogonal
    rotation (|Q - 1|_F ~ eps, as in small_rotations) of the previous one,
    starting from a Haar-random state: the near-linearly-dependent ansatz that
    rank growing (Sec. III.C) produces, with an ill-conditioned Gram matrix."""
    n = 2 * N
    out = np.empty((R, n, n))
    out[0] = random_states(N, 1, seed=seed)[0]
    rots = small_rotations(n, R - 1, eps, seed=seed + 1)
    for mu in range(1, R):
        g = rots[mu - 1] @ out[mu - 1] @ rots[mu - 1].T
        out[mu] = 0.5 * (g - g.T)
    return out
