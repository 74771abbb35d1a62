"""Model Hamiltonians and observables in Majorana form.

Conventions (the paper leaves the Majorana-to-mode map unstated, Sec. II.A):

* ``2N`` Majoranas ``c_0 .. c_{2N-1}`` with ``{c_j, c_k} = 2 delta_jk``.
* Fermion mode ``j`` is ``a_j = (c_{2j} + i c_{2j+1}) / 2``; the vacuum then has
  covariance matrix ``Gamma_0 = (+) [[0, 1], [-1, 0]]``.
* ``H = e0 + H_2 + H_4`` with ``H_2 = i sum_{k,l} A_kl c_k c_l`` (both index
  orders summed, ``A`` real skew) and ``H_4 = sum_q u_q c_a c_b c_c c_d`` over
  sorted quadruples ``a<b<c<d``; the fully antisymmetric tensor of Sec. II.A is
  ``U = u / 24`` on every ordering of the quadruple.

A fermionic operator is described as a list of terms ``(coef, ops)`` where
``ops`` is a tuple of ``(mode, dagger)`` factors applied left to right.  The
converter expands every factor into Majoranas and brings each word to sorted
order with the anticommutation sign, using ``c_k c_k = 1``.  This is algebra of
the problem statement, not of the SGS method.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, Iterable, List, Sequence, Tuple

import numpy as np

Word = Tuple[int, ...]
FermionTerm = Tuple[complex, Tuple[Tuple[int, bool], ...]]


def _normal_order(word: Sequence[int]) -> Tuple[int, Word]:
    """Sort a Majorana word; return (sign, reduced sorted word)."""
    w = list(word)
    sign = 1
    # insertion sort, counting transpositions of distinct neighbours
    for i in range(1, len(w)):
        j = i
        while j > 0 and w[j - 1] > w[j]:
            w[j - 1], w[j] = w[j], w[j - 1]
            sign = -sign
            j -= 1
    # cancel equal neighbours: c_k c_k = 1
    out: List[int] = []
    for k in w:
        if out and out[-1] == k:
            out.pop()
        else:
            out.append(k)
    return sign, tuple(out)


class MajoranaPoly(dict):
    """A polynomial in Majoranas: {sorted distinct word: complex coefficient}."""

    def add(self, word: Word, coef: complex) -> None:
        if coef == 0:
            return
        self[word] = self.get(word, 0.0) + coef

    def cleaned(self, tol: float = 1e-14) -> "MajoranaPoly":
        out = MajoranaPoly()
        for w, c in self.items():
            if abs(c) > tol:
                out[w] = complex(c)
        return out

    def __mul__(self, other: "MajoranaPoly") -> "MajoranaPoly":
        out = MajoranaPoly()
        for w1, c1 in self.items():
            for w2, c2 in other.items():
                s, w = _normal_order(w1 + w2)
                out.add(w, s * c1 * c2)
        return out

    def scaled(self, f: complex) -> "MajoranaPoly":
        out = MajoranaPoly()
        for w, c in self.items():
            out[w] = c * f
        return out

    def __add__(self, other: "MajoranaPoly") -> "MajoranaPoly":
        out = MajoranaPoly(self)
        for w, c in other.items():
            out.add(w, c)
        return out

    def degree(self) -> int:
        return max((len(w) for w in self), default=0)


def _fermion_op(mode: int, dagger: bool) -> MajoranaPoly:
    p = MajoranaPoly()
    p[(2 * mode,)] = 0.5
    p[(2 * mode + 1,)] = -0.5j if dagger else 0.5j
    return p


def fermion_terms_to_majorana(terms: Iterable[FermionTerm]) -> MajoranaPoly:
    """Expand fermionic operator products into a Majorana polynomial."""
    total = MajoranaPoly()
    for coef, ops in terms:
        prod = MajoranaPoly({(): complex(coef)})
        for mode, dag in ops:
            prod = prod * _fermion_op(mode, dag)
        total = total + prod
    return total.cleaned()


@dataclass
class MajoranaHamiltonian:
    """H = e0 + i sum A_kl c_k c_l + sum_q u_q c_{q0} c_{q1} c_{q2} c_{q3}
    + sum_w h_w c_{w0} ... c_{w(m-1)} over words of m = 6 or 8 Majoranas.

    A Hermitian word term has h_w = v_w i^((m/2) mod 2) with v_w real (the
    reversed word is (-1)^(m(m-1)/2) times the word): imaginary for m = 6,
    real for m = 8.  ``higher_val`` holds v_w.
    """

    N: int
    A: np.ndarray  # (2N, 2N) real skew, float64
    quartic_idx: np.ndarray  # (nq, 4) int32, each row strictly increasing
    quartic_val: np.ndarray  # (nq,) float64
    e0: float
    meta: Dict[str, object] = field(default_factory=dict)
    higher_idx: Tuple[Tuple[int, ...], ...] = ()  # words of 6 or 8 indices, strictly increasing
    higher_val: np.ndarray = field(default_factory=lambda: np.zeros(0))  # (nw,) float64, v_w

    @staticmethod
    def word_phase(m: int) -> complex:
        """h_w / v_w for a Hermitian word term of m Majoranas."""
        return 1j if (m // 2) % 2 else 1.0

    @property
    def n(self) -> int:
        return 2 * self.N

    @staticmethod
    def from_poly(N: int, poly: MajoranaPoly, tol: float = 1e-13) -> "MajoranaHamiltonian":
        n = 2 * N
        A = np.zeros((n, n))
        qi: List[Word] = []
        qv: List[float] = []
        hi: List[Word] = []
        hv: List[float] = []
        e0 = 0.0
        for w, c in sorted(poly.items()):
            if len(w) == 0:
                if abs(c.imag) > tol:
                    raise ValueError("non-Hermitian constant")
                e0 += c.real
            elif len(w) == 2:
                # c * c_k c_l (k<l) == i (A_kl c_k c_l + A_lk c_l c_k) = 2i A_kl c_k c_l
                a = c / 2j
                if abs(a.imag) > tol:
                    raise ValueError("non-Hermitian quadratic term %r" % (w,))
                k, l = w
                A[k, l] += a.real
                A[l, k] -= a.real
            elif len(w) == 4:
                if abs(c.imag) > tol:
                    raise ValueError("non-Hermitian quartic term %r" % (w,))
                qi.append(w)
                qv.append(c.real)
            elif len(w) in (6, 8):
                v = c / MajoranaHamiltonian.word_phase(len(w))
                if abs(v.imag) > tol:
                    raise ValueError("non-Hermitian term %r" % (w,))
                hi.append(tuple(int(x) for x in w))
                hv.append(v.real)
            else:
                raise ValueError("term of degree %d is not supported" % len(w))
        return MajoranaHamiltonian(
            N=N,
            A=A,
            quartic_idx=np.array(qi, dtype=np.int32).reshape(-1, 4),
            quartic_val=np.array(qv, dtype=np.float64),
            e0=float(e0),
            higher_idx=tuple(hi),
            higher_val=np.array(hv, dtype=np.float64),
        )

    def poly(self) -> MajoranaPoly:
        """Back to a Majorana polynomial (used by checks)."""
        p = MajoranaPoly()
        if self.e0:
            p[()] = complex(self.e0)
        n = self.n
        for k in range(n):
            for l in range(k + 1, n):
                if self.A[k, l] != 0.0:
                    p.add((k, l), 2j * self.A[k, l])
        for w, u in zip(self.quartic_idx, self.quartic_val):
            p.add(tuple(int(x) for x in w), complex(u))
        for w, v in zip(self.higher_idx, self.higher_val):
            p.add(tuple(w), v * self.word_phase(len(w)))
        return p

    def impurity_majoranas(self) -> np.ndarray:
        """Sorted Majorana indices touched by the interaction words (the M of Sec. II.A)."""
        idx = [int(x) for x in self.quartic_idx.reshape(-1)] + [x for w in self.higher_idx for x in w]
        return np.unique(np.array(idx, dtype=np.int64)).astype(np.int32)


# ---------------------------------------------------------------------------
# single-impurity Anderson model (Sec. IV): impurity site 0, chain sites 1..L
# ---------------------------------------------------------------------------

def siam_mode(site: int, spin: int) -> int:
    """Mode index of (site, spin); site 0 is the impurity, spin 0 = up."""
    return 2 * site + spin


def _hop(coef: float, i: int, j: int) -> List[FermionTerm]:
    """coef * (a_i^dag a_j + a_j^dag a_i)."""
    return [(coef, ((i, True), (j, False))), (coef, ((j, True), (i, False)))]


def _num(coef: float, i: int) -> List[FermionTerm]:
    return [(coef, ((i, True), (i, False)))]


def anderson_terms(L: int, U: float, V: float, t: float = 1.0,
                   eps_d: float | None = None, mu: float = 0.0,
                   wilson_tail: Sequence[float] = ()) -> Tuple[int, List[FermionTerm]]:
    """Fermionic terms of the SIAM on a chain with L bath sites per spin.

    H = -V sum_s (d0s^dag d1s + h.c.) - t sum_{r=1}^{L-1} sum_s (d_rs^dag d_{r+1}s + h.c.)
        + eps_d n_0 + U n_0up n_0dn - mu sum_{r>=1} n_r
    ``wilson_tail`` appends extra sites with the given hoppings (Fig. 4 caption).
    """
    if eps_d is None:
        eps_d = -U / 2.0
    nsites = 1 + L + len(wilson_tail)
    N = 2 * nsites
    terms: List[FermionTerm] = []
    hops = [V] + [t] * (L - 1) + list(wilson_tail)
    for r, h in enumerate(hops):
        for s in (0, 1):
            terms += _hop(-h, siam_mode(r, s), siam_mode(r + 1, s))
    for s in (0, 1):
        terms += _num(eps_d, siam_mode(0, s))
    if U != 0.0:
        terms.append((U, ((siam_mode(0, 0), True), (siam_mode(0, 0), False),
                          (siam_mode(0, 1), True), (siam_mode(0, 1), False))))
    if mu != 0.0:
        for r in range(1, nsites):
            for s in (0, 1):
                terms += _num(-mu, siam_mode(r, s))
    return N, terms


def anderson_multibody_terms(L: int, U: float, V: float, W3: float, W4: float,
                             t: float = 1.0) -> Tuple[int, List[FermionTerm]]:
    """The Anderson chain plus density interactions of three and four bodies
    between the impurity and the first bath site,
      W3 n_0up n_0dn n_1up + W4 n_0up n_0dn n_1up n_1dn,
    which give Majorana words of 6 and 8 operators (interaction terms of
    weight m > 4, Sec. III.C).  A synthetic model: the paper names no such
    Hamiltonian."""
    N, terms = anderson_terms(L, U, V, t)
    n = lambda site, spin: ((siam_mode(site, spin), True), (siam_mode(site, spin), False))
    if W3 != 0.0:
        terms.append((W3, n(0, 0) + n(0, 1) + n(1, 0)))
    if W4 != 0.0:
        terms.append((W4, n(0, 0) + n(0, 1) + n(1, 0) + n(1, 1)))
    return N, terms


def anderson_multibody(L: int, U: float, V: float, W3: float, W4: float, t: float = 1.0) -> MajoranaHamiltonian:
    N, terms = anderson_multibody_terms(L, U, V, W3, W4, t)
    h = MajoranaHamiltonian.from_poly(N, fermion_terms_to_majorana(terms))
    h.meta = dict(model="anderson_multibody", L=L, U=U, V=V, W3=W3, W4=W4, t=t)
    return h


def wilson_hoppings(L_W: int = 20, Lambda: float = 1.2, t: float = 1.0) -> List[float]:
    """Hoppings t_n = Lambda^-n t, n = 1..L_W, of the tail appended to the bath
    to reduce finite-size effects (Fig. 4 caption: L_W = 20, Lambda = 1.2)."""
    return [t * Lambda ** (-k) for k in range(1, L_W + 1)]


def anderson(L: int, U: float, V: float, t: float = 1.0, eps_d: float | None = None,
             mu: float = 0.0, wilson_tail: Sequence[float] = ()) -> MajoranaHamiltonian:
    N, terms = anderson_terms(L, U, V, t, eps_d, mu, wilson_tail)
    h = MajoranaHamiltonian.from_poly(N, fermion_terms_to_majorana(terms))
    h.meta = dict(model="anderson", L=L, U=U, V=V, t=t,
                  eps_d=(-U / 2.0 if eps_d is None else eps_d), mu=mu)
    return h


# ---------------------------------------------------------------------------
# spin operators and the two-channel Kondo model (Sec. V)
# ---------------------------------------------------------------------------

_PAULI = {
    "x": np.array([[0, 1], [1, 0]], dtype=complex),
    "y": np.array([[0, -1j], [1j, 0]], dtype=complex),
    "z": np.array([[1, 0], [0, -1]], dtype=complex),
}


def spin_dot_terms(modes_a: Tuple[int, int], modes_b: Tuple[int, int],
                   coef: float = 1.0) -> List[FermionTerm]:
    """coef * S_a . S_b with S = 1/2 sum_{ss'} d_s^dag sigma_{ss'} d_s'.

    ``modes_a`` / ``modes_b`` are the (up, down) mode indices of the two sites.
    """
    terms: List[FermionTerm] = []
    for comp in "xyz":
        s = _PAULI[comp]
        for s1 in range(2):
            for s2 in range(2):
                if s[s1, s2] == 0:
                    continue
                for s3 in range(2):
                    for s4 in range(2):
                        if s[s3, s4] == 0:
                            continue
                        c = coef * 0.25 * s[s1, s2] * s[s3, s4]
                        terms.append((c, ((modes_a[s1], True), (modes_a[s2], False),
                                          (modes_b[s3], True), (modes_b[s4], False))))
    return terms


def spin_dot_poly(modes_a: Tuple[int, int], modes_b: Tuple[int, int]) -> MajoranaPoly:
    return fermion_terms_to_majorana(spin_dot_terms(modes_a, modes_b))


def tck_mode(channel: int | None, site: int, spin: int, L: int) -> int:
    """Mode index in the two-channel Kondo layout: impurity = modes 0, 1;
    channel c (0 or 1), site r (0..L-1): 2 + 2 * (c * L + r) + spin."""
    if channel is None:
        return spin
    return 2 + 2 * (channel * L + site) + spin


def two_channel_kondo_terms(L: int, J: float, U: float = 8.0, eps_d: float | None = None,
                            t: float = 1.0) -> Tuple[int, List[FermionTerm]]:
    """Fermionic impurity with large U (single occupancy), coupled by J S_imp . S_c(0)
    to site 0 of two independent spinful chains of L sites each."""
    if eps_d is None:
        eps_d = -U / 2.0
    N = 2 + 2 * 2 * L
    terms: List[FermionTerm] = []
    for c in (0, 1):
        for r in range(L - 1):
            for s in (0, 1):
                terms += _hop(-t, tck_mode(c, r, s, L), tck_mode(c, r + 1, s, L))
    for s in (0, 1):
        terms += _num(eps_d, tck_mode(None, 0, s, L))
    terms.append((U, ((0, True), (0, False), (1, True), (1, False))))
    imp = (tck_mode(None, 0, 0, L), tck_mode(None, 0, 1, L))
    for c in (0, 1):
        site0 = (tck_mode(c, 0, 0, L), tck_mode(c, 0, 1, L))
        terms += spin_dot_terms(imp, site0, coef=J)
    return N, terms


def two_channel_kondo(L: int, J: float, U: float = 8.0, eps_d: float | None = None,
                      t: float = 1.0) -> MajoranaHamiltonian:
    N, terms = two_channel_kondo_terms(L, J, U, eps_d, t)
    h = MajoranaHamiltonian.from_poly(N, fermion_terms_to_majorana(terms))
    h.meta = dict(model="two_channel_kondo", L=L, J=J, U=U,
                  eps_d=(-U / 2.0 if eps_d is None else eps_d), t=t)
    return h
