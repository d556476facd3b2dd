"""Plain FP64 CPU oracle for the collocation interior-point Newton step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's CPU
baseline leg may import this package.  It shares no code with the GPU library: it has its
own collocation tables, its own problem functions and derivatives, its own KKT algebra
(dense unreduced LDL^T for parity, natural-order block Cholesky for timing) and its own
interior-point loop.  Everything is written from the paper's problem statement (eq. 1-3)
and from the published filter line-search interior-point method it names (Waechter &
Biegler, Math. Prog. 106, 2006), step by step and without blocking or reordering beyond
what those definitions state.

Modules
  tables   collocation nodes and Lagrange weights (eq. 2b-2c, eq. 3)
  problem  constraints, objective and their first/second derivatives (eq. 2)
  kkt      relaxed-equality primal-dual system: unreduced and condensed forms
  blocksolve  natural-order block-tridiagonal-with-border Cholesky of the condensed matrix
  ipm      filter line-search interior-point iteration
"""
