"""CPU FP64 oracle for the multilevel quasidiffusion (MLQD) method with multigrid
in photon frequency (Anistratov, arXiv 2011.05427).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously-correct
reference that the GPU library is checked against.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the GPU
product path never calls it and shares no code with it.

Modules (each function cites the passage of the paper it follows):
  planck   group Planck integrals B_g(T), dB_g/dT and the point opacity law
  sweep    simple corner balance transport sweep (Sec. 5, implicit Euler)
  moments  QD (Eddington) factors and boundary factors (Eqs. f_g, c_g, mloqd-bcs)
  lo       discrete low-order QD equations at one frequency level (Eqs. mloqd-d,
           mloqd-d-gamma) and the grey level coupled to the MEB (Eq. eb-Gamma-d)
  restrict restriction of coefficients to coarser frequency grids
           (Eqs. coeff-gamma, g-notation, eta-gamma, coeff-Gamma, eta-Gamma)
  mlqd     time stepping (Alg. 3, with Alg. 2 as its V-cycle case)
  mlp      FP64 reference of the learned closure network (forward/backward)

Parity status: every function is pinned by CPU tests against closed forms,
invariants, brute force or library routines, except the transient multi-step
profiles (the paper prints no solution values), whose parity is unpinned beyond
the invariants checked in tests.
"""
