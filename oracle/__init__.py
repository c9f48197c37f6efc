"""Plain, slow, FP64 CPU oracle for the PBM + multigrid-MINRES method of
Brune & Kocvara, "On barrier and modified barrier multigrid methods for 3d
topology optimization" (arXiv 1904.06556).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check of
the entry module and the CPU-baseline leg of the benchmark may import it.  The
product path (the HIP library and its Python binding) never calls into it and
shares no code with it: every formula here is written out from the paper with
NumPy/SciPy, each function citing the passage it follows.

Modules
  fe       hexahedral Q1 element stiffness, grids, assembly, K(rho) x,
           element energies (Section 1 eq. (1.1); Section 6.2)
  penalty  the penalty-barrier function phi with tau_hat = -1/2 (Section 3.1)
  pbm      augmented Lagrangian of the dual VTS problem, its gradient and
           Hessian, the Schur complement S, the reduced Newton system, the
           Newton method (Algorithm 2) and the PBM outer loop (Algorithm 1)
  mg       trilinear prolongation, Galerkin coarse operators, multicolour
           block Gauss-Seidel, the V-cycle (Section 6.1)
  minres   preconditioned MINRES (Section 6.1)
  kkt      compliance, KKT residual and the duality certificate (Section 2)
  doc      damped optimality criteria, the comparison method (Section 5,
           Algorithm 4)
  ip       primal-dual interior point method, the other comparison method
           (Section 4, Algorithm 3)

Parity status: every function is pinned by a `-m "not gpu"` test except where
its docstring says "parity unpinned".
"""
