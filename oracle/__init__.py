"""CPU oracle for the steady-state solver -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct reference implementations of what the solver
computes, written from the paper (Nation, "Steady-state solution methods for
open quantum optical systems"):

  liouvillian  eq. (lindblad) with column-stacking vectorisation, eq. (eigval)
  steady       eq. (linear): unit-trace row, solved by dense LU (fp64)
  ordering     bandwidth and profile definitions (section "Direct
               factorization"), Cuthill-McKee / reverse Cuthill-McKee on the
               symmetrised pattern of the matrix
  ilu          incomplete LU with zero fill, ILU(0), and the dual-threshold
               ILUT of the section "Iterative Solvers"
  invariants   Hermiticity, trace, positivity and residual checks

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU path and never calls it.
"""
