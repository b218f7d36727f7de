"""FP64 CPU oracle for the monodomain time step.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The HIP library never calls it and shares no code with
it: the two sides are written independently from the paper and meet only on
the seeded inputs of the `workloads` module.

Layout
  fem.py        finite-element mass and stiffness (Section "Cardiac
                electrophysiology: numerical discretization", eq. of the
                linear system and the definitions of M, K that follow it)
  ionic.py      the ionic models (eq. of the ionic model ODEs) with the
                Rush-Larsen / explicit integrator
  monodomain.py BDF/IMEX time stepping with ionic current interpolation,
                linear solvers and activation times
  cell.py       single-cell pacing (the monodomain step without diffusion)

Parity status per function is stated in each module header; every function
listed there is pinned by a `-m "not gpu"` test unless marked
"parity unpinned".
"""
from . import cell, fem, ionic, monodomain  # noqa: F401
