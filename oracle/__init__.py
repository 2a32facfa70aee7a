"""CPU FP64 oracle for the Woodbury-preconditioned Gauss-Newton linear solve.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the benchmark's CPU
baseline leg use it. It shares no code with the HIP library; the two sides meet
only in the seeded input generators (package h1w_inputs), which hold none of
the method's arithmetic.

Everything here is plain numpy/scipy in float64, written for a reader to check
against the paper by eye, with no blocking, fusion or reordering beyond what the
definitions state:

  operator   the discrete H^1 Gram operator A = K + beta*M (structured grid,
             Neumann boundary) and its lumped mass W            (module operator)
  poisson    exact A^{-1} by the DCT-I eigen-decomposition; sparse LU  (poisson)
  multigrid  a textbook symmetric V-cycle B ~ A^{-1} with the same parameters as
             the GPU's (the Poisson solver inside the preconditioner) (multigrid)
  gn         the GN system (alpha*A + J^T J) x = b by three independent routes,
             the paper's right-hand side and closed-form update, and the
             Woodbury preconditioner apply                          (gn)
  ert        the ERT forward map of Section 4 on the structured grid: the
             conductance operator, pole fields by sparse LU, pole-pole
             voltages and their sensitivities by the adjoint formula  (ert)

Each function names the passage of Blechta & Ernst (arXiv 2209.02815) it
follows. Pins (closed forms, invariants, special cases, brute force) live in
tests/test_oracle_*.py; no function here is "parity unpinned".
"""
from . import operator, poisson, multigrid, gn, ert  # noqa: F401
