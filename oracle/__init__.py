"""FP64 CPU oracle for the MF-CIM L0RBCS solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
statement of what the solver computes, written from the paper's equations.
Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import it; the GPU library and its Python binding never do, and the two share
no code (the seeded input generators in ``workloads`` are the only common
dependency, and they hold none of the solver's arithmetic).

Modules:
  mfcim  - schedules, couplings, fields, Euler integration, CDP, Algorithm 1
  brute  - exhaustive optimum of eq. 3 and eq. 4 for N <= 16
  rng    - counter-based SplitMix64 + Box-Muller initial amplitudes
  mri    - the MRI-shaped measurement operator (orthonormal DCT-II and Haar)

Pinned by tests/test_oracle_*.py against closed forms, brute force,
published generator outputs and textbook least squares; see each test's
docstring for what it fixes.
"""
from . import brute, mfcim, rng  # noqa: F401
from .mfcim import BN, CN, CimParams, OuterParams  # noqa: F401
