"""Pfaffians of skew-symmetric matrices (real or complex).

The paper evaluates Pfaffians numerically (acknowledgments) without stating the
algorithm.  The oracle uses two independent definitions:

* ``pfaffian_expand``: the defining expansion along the first row,
  Pf(A) = sum_j (-1)^(j+1) a_0j Pf(A with rows/cols 0, j removed)
  (exponential cost, used for tiny pins only);
* ``pfaffian_log``: elimination with 2x2 pivot blocks.  For a skew matrix
  written as [[P, B], [-B^T, D]] with P = [[0, a], [-a, 0]],
  Pf = a * Pf(D + B^T P^{-1} B); before each elimination the largest entry of
  the first column is moved to row/column 1 by a symmetric swap, which flips
  the sign of the Pfaffian.

Both return exact results up to rounding; tests pin them against each other,
against Pf^2 = det and against Pf(Q^T A Q) = det(Q) Pf(A).
"""

from __future__ import annotations

import cmath
import math
from typing import Tuple

import numpy as np


def pfaffian_expand(a: np.ndarray) -> complex:
    a = np.asarray(a)
    n = a.shape[0]
    if n == 0:
        return 1.0
    if n % 2:
        return 0.0
    total = 0.0
    idx = list(range(1, n))
    for pos, j in enumerate(idx):
        rest = [k for k in idx if k != j]
        sub = a[np.ix_(rest, rest)]
        total += (-1) ** pos * a[0, j] * pfaffian_expand(sub)
    return total


def pfaffian_log(a: np.ndarray) -> Tuple[float, complex]:
    """Return (log|Pf(a)|, Pf(a)/|Pf(a)|); (-inf, 0) for a singular matrix."""
    m = np.array(a, dtype=complex if np.iscomplexobj(a) else float, copy=True)
    n = m.shape[0]
    if n % 2:
        return -math.inf, 0.0
    logabs = 0.0
    phase: complex = 1.0
    for k in range(0, n - 1, 2):
        # pivot: largest |m[i, k]| for i > k, brought to row/col k+1
        col = np.abs(m[k + 1:, k])
        p = k + 1 + int(np.argmax(col))
        if p != k + 1:
            m[[k + 1, p], :] = m[[p, k + 1], :]
            m[:, [k + 1, p]] = m[:, [p, k + 1]]
            phase = -phase
        piv = m[k, k + 1]
        if piv == 0:
            return -math.inf, 0.0
        logabs += math.log(abs(piv))
        phase *= piv / abs(piv)
        if k + 2 < n:
            b0 = m[k, k + 2:].copy()      # row k of the trailing block
            b1 = m[k + 1, k + 2:].copy()  # row k+1
            # D + B^T P^{-1} B with P^{-1} = [[0, -1/a], [1/a, 0]]
            upd = (np.outer(b1, b0) - np.outer(b0, b1)) / piv
            m[k + 2:, k + 2:] += upd
    return logabs, phase


def pfaffian(a: np.ndarray) -> complex:
    la, ph = pfaffian_log(a)
    if la == -math.inf:
        return 0.0
    v = ph * math.exp(la)
    if not np.iscomplexobj(a):
        return float(np.real(v))
    return complex(v)


def phase_of(z: complex) -> float:
    return cmath.phase(z)
