"""Seeded synthetic inputs shared by the HIP path and the CPU oracle.

This package builds the *inputs* of the SGS imaginary-time step and nothing
else: model Hamiltonians written in Majorana form (Sec. II.A of Boutin & Bauer,
arXiv:2105.01088), observables written the same way, and seeded Haar-random
initial covariance matrices.  It holds none of the method's arithmetic (no
overlaps, Wick contractions, amplitude solves or forces), so that the two sides
it feeds stay independent.
"""

from .models import (  # noqa: F401
    MajoranaPoly,
    MajoranaHamiltonian,
    fermion_terms_to_majorana,
    anderson_terms,
    anderson,
    anderson_multibody_terms,
    anderson_multibody,
    two_channel_kondo_terms,
    two_channel_kondo,
    spin_dot_terms,
    spin_dot_poly,
    siam_mode,
    wilson_hoppings,
)
from .states import vacuum_cm, haar_so, random_states, small_rotations, near_copy_states  # noqa: F401
from .configs import CONFIGS, config_problem, batched_problems  # noqa: F401
