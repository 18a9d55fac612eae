"""CPU FP64 oracle for the implicit phase-field hot path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check of the entry
module and the CPU-baseline leg of the benchmark may import this package.  The
product path (the HIP library and its Python binding) never imports, calls or
links anything here, and nothing here imports the product path.

It is a plain, slow, direct transcription of the discrete method written from
the paper (Ghosh, Newman, Francois, "Tusas: a fully implicit parallel approach
for coupled phase-field equations"):

* fem      -- Q1 box mesh, 3-point Gauss rule, the coupled residual F(phi, u)
              (Sec. 2.1.1-2.1.2; phi equation Eq. pf2 / lambda with k = 1, thermal
              equation Eq. dtemp / temp1, anisotropy Eq. gs)
* deriv    -- complex-step Jacobians, Jv, VJP and parameter derivatives
              (Jacobian definition of Sec. 2.2)
* precond  -- the block-diagonal preconditioner of Sec. 2.3.2 (Eqs. pre, m11,
              m22, pref2, preconc2) with its geometric-multigrid inverse
* solvers  -- exact-Jacobian Newton with the backtracking of Eq. glob and the
              termination test of Eq. tolerance; backward-Euler stepping; the
              discrete adjoint of the stepping

Parity status of every function is stated in its docstring and in the design
notes; functions with no independent pin say "parity unpinned".
"""
