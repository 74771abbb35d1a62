"""Exact diagonalization in the even-parity sector.

Gaussian states reached from the vacuum by SO(2N) rotations keep Pf(Gamma) = +1,
i.e. even fermion parity, so the variational energies are bounded below by the
lowest even-parity eigenvalue.  The Hamiltonian is built from the fermionic
terms directly (Jordan-Wigner), independently of the Majorana conversion.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fock import fermion_operator_sparse


def even_sector_ground_energy(N: int, terms) -> float:
    H = fermion_operator_sparse(N, terms)
    dim = 2 ** N
    occ = np.array([bin(x).count("1") for x in range(dim)])
    even = np.nonzero(occ % 2 == 0)[0]
    He = H[even][:, even]
    He = 0.5 * (He + He.conj().T)
    if len(even) <= 512:
        return float(np.linalg.eigvalsh(He.toarray())[0])
    w = spla.eigsh(He.tocsr(), k=1, which="SA", tol=1e-13, return_eigenvectors=False)
    return float(np.min(w).real)
