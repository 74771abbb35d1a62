"""CPU FP64 oracle for the SGS imaginary-time step (Boutin & Bauer, arXiv:2105.01088).

TEST INFRASTRUCTURE ONLY.  This package is imported by ``tests/``, by the
smoke check in ``__graft_entry__`` and by the ``cpu_baseline`` leg of
``bench.py``; the product path never imports, links or runs it.  It shares no
code with the HIP library: its only common dependency is ``sgs_inputs``, which
builds seeded inputs and holds none of the method's arithmetic.

Everything here is plain numpy/scipy in float64, written for a reader to check
against the paper by eye: no blocking, fusion or reordering beyond what the
cited definition or algorithm states.

Modules
  pfaffian     Pfaffians (Parlett-Reid elimination, and brute-force expansion)
  fock         Jordan-Wigner Fock-space matrices for brute-force pins (N <= 8)
  gaussian     overlaps with phase, transition matrices, generalized Wick
  sgs          amplitude solve, equations of motion, Euler step + purification
  observables  correlation functions and the Renyi-2 entropy
  ed           exact diagonalization in the even-parity sector
"""
