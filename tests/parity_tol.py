"""Covariance-matrix tolerance for the printed weights, shared by the GPU
parity tests.

With printed weights the force on state mu carries lambda_b / lambda_mu.  A
backward-stable eigen-solver returns lambda with componentwise error
delta <= R eps |lambda| |X|^2 (|h| + |E| |G|) / gap, with X the canonical
basis (X^dag G X = 1) and gap the distance from E to the next root of the
projected problem; the ratio then carries a relative error of about
2 delta / |lambda_mu|, and so does the force on mu.  States at or below the
amplitude floor (1e-13 max|lambda|) keep only their exact self term."""

import numpy as np

from oracle import sgs as osgs

EPS = np.finfo(float).eps


def printed_tol(ref, dtau, base=1e-10):
    """(per-state tolerance, per-state amplification 2 delta / |lambda_mu|) for
    the states stepped by ref (an oracle StepResult) with step dtau.  The same
    bound covers the unit-modulus weight, whose factor
    |lambda~_mu| (lambda_mu^* / |lambda_mu|) lambda_b has the same sensitivity to
    the phase of lambda_mu."""
    G, h = ref.tables.G, ref.tables.h
    R = G.shape[0]
    X = osgs.canonical_basis(G)
    hp = X.conj().T @ (0.5 * (h + h.conj().T)) @ X
    ev = np.linalg.eigvalsh(0.5 * (hp + hp.conj().T))
    gap = ev[1] - ev[0] if ev.shape[0] > 1 else abs(ev[0])
    lam = np.abs(ref.lam)
    delta = R * EPS * np.linalg.norm(ref.lam) * np.linalg.norm(X, 2) ** 2 * \
        (np.linalg.norm(h, 2) + abs(ref.E) * np.linalg.norm(G, 2)) / gap
    amp = np.where(lam > osgs.LAMBDA_FLOOR * lam.max(), 2 * delta / np.maximum(lam, 1e-300), 0.0)
    dmax = np.abs(ref.dgamma).reshape(R, -1).max(axis=1)
    return base + dtau * dmax * amp, amp


def energy_tol(ref, base=1e-10):
    """Relative energy tolerance: base, plus the energy error that a
    backward error R eps (|h| + |E| |G|) in h and G produces for an amplitude
    vector normalized lambda^dag G lambda = 1: R eps |lambda|^2 (|h| + |E| |G|)
    / |E| (cond(G) eps when G is ill-conditioned)."""
    G, h = ref.tables.G, ref.tables.h
    R = G.shape[0]
    lam2 = np.linalg.norm(ref.lam) ** 2
    return base + R * EPS * lam2 * (np.linalg.norm(h, 2) + abs(ref.E) * np.linalg.norm(G, 2)) / abs(ref.E)


def phase_tol(g0, ga_, gb, base=1e-9, factor=16.0):
    """Tolerance on exp(i arg) of a Gram-matrix entry computed through the
    Schur-reduced triple product (Sec. II.B): its phase is that of Pf(C_ab),
    C_ab = i (G_b + G_0) - i X_a.  To first order a perturbation changes
    ln Pf(C) by tr(C^-1 dC) / 2, at most kappa(C) / 2 times the relative
    perturbation of C; a GPU C_ab carries a few ulps per entry (from the
    products that form X_a).  factor covers that count with margin:
    measured errors at n = 800 and 1204 stay 3-15 times below
    factor kappa(C) eps on both Gauss-Jordan variants."""
    from oracle import gaussian as ga
    s = np.linalg.svd(ga.schur_matrix(g0, ga_, gb), compute_uv=False)
    return max(base, factor * (s[0] / s[-1]) * EPS)
