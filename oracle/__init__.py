"""Plain, slow, FP64 CPU oracle for the kLST generalized eigenproblem.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check of the graft
entry point and the CPU-baseline leg of the benchmark may import anything in
this package; the product path (the native library and its Python binding)
never does, and shares no code with it.

Modules
  grid       -- Chebyshev-Gauss-Lobatto nodes, differentiation matrix, algebraic
                map (Sec. 3.1, eqs. ChebPoints, ChebDiag, ChebOffDiag, ChebBC,
                Chebmapping).
  velocity   -- Gauss-Hermite nodes/weights by Golub-Welsch (Sec. 3.2).
  operator   -- base macros, equilibria, linearisation coefficients and the
                explicit pencil (A, B) (Sec. 2.2, eqs. CompBGKtilde, Comp1DHarm,
                comp_ghat1Dshock, comp_hhat1Dshock, MatrixSystem).
  eig        -- the result definition: finite eigenvalues of (A, B) nearest a
                target, by dense QZ (Sec. 4, eq. MatrixProblem) and by exact
                shift-invert Arnoldi with a structured (Woodbury) inverse.
  jd         -- a plain Jacobi-Davidson (harmonic extraction, partial Schur
                deflation, block-Jacobi preconditioned GMRES correction) following
                the steps of Sec. 4.2; the CPU baseline.
  parity     -- the eigenpair matching rule used by the parity tests.
  bgk        -- BE-BGK base-flow relaxation: MUSCL-minmod finite volumes on the
                mapped nodes, BGK collision, RK4 in time (Sec. 3.3).
  post       -- macroscopic perturbations of eigenvectors and |U_hat| (Sec. 2.2,
                Sec. 5 eq. Unormpert); the base flow's non-equilibrium level
                (Sec. 5, eq. L2norm).
"""
