"""Plain FP64 CPU oracle for the coupled Stokes-Darcy solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only the test-suite, the package's smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP library; both sides
receive the same seeded inputs from :mod:`sdinputs`.

Modules
  assemble  staggered finite-volume Stokes + two-point-flux Darcy + interface
            rows (Sec. 2, eqs. for momentum, Darcy and the three coupling
            conditions; block structure of the pv formulation)
  direct    sparse LU reference solve (the plain definition x* = A^-1 b)
  dn        partitioned Dirichlet-Neumann fixed point with Aitken relaxation
            or IQN-ILS (Sec. 3, fixed-point problem and stopping rule)
  amg       aggregation AMG setup and V-cycle (Sec. 5 solver setup)
  precond   pressure-velocity block-Jacobi / block-Gauss-Seidel (Sec. 4)
  krylov    FGMRES(m) with classical Gram-Schmidt twice, PD-GMRES (restart
            lengths from a proportional-derivative controller), BiCGSTAB,
            and the mixed-precision iterative-refinement driver
  ilu       ILU(0) of the Darcy block and its triangular solves (Table 2's
            ILU rows)
  hashing   the 32-bit integer finaliser used for aggregation priorities
  transient backward-Euler steps of the transient free flow (Sec. 2)
  assemble3d the same model and closures on a 3-D box grid
"""
