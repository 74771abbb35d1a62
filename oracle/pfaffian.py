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
from scipy.linalg import blas


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
    cplx = np.iscomplexobj(a)
    m = np.array(a, dtype=complex if cplx else float, copy=True, order="C")
    geru = blas.zgeru if cplx else blas.dger
    n = m.shape[0]
    if n % 2:
        return -math.inf, 0.0
    logabs = 0.0
    phase: complex = 1.0
    for k in range(0, n - 1, 2):
        # pivot: largest |m[i, k]| for i > k, brought to row/col k+1
        p = k + 1 + int(np.argmax(np.abs(m[k + 1:, k])))
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
            # trailing block D + B^T P^{-1} B, P^{-1} = [[0, -1/a], [1/a, 0]]:
            # D += (b1 b0^T - b0 b1^T) / a, with b0 = row k, b1 = row k+1;
            # applied as two in-place BLAS rank-1 updates of the trailing rows
            # (columns left of k+2 receive zeros).
            b0 = np.zeros(n, dtype=m.dtype)
            b1 = np.zeros(n, dtype=m.dtype)
            b0[k + 2:] = m[k, k + 2:]
            b1[k + 2:] = m[k + 1, k + 2:]
            rows = m[k + 2:, :].T  # column-major view of rows k+2.., updated in place
            geru(1.0 / piv, b0, b1[k + 2:], a=rows, overwrite_a=1)
            geru(-1.0 / piv, b1, b0[k + 2:], a=rows, overwrite_a=1)
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
