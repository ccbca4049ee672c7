"""Plain, slow CPU FP64 oracle of the implicit DG Navier-Stokes hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package; the device library
never does, and this package never imports the device library.

It follows arxiv 2002.04222 ("Implicit ... Nektar++ ... compressible
flow solver"), written from the paper:

  basis.py    orthonormal tensor Legendre basis, Gauss quadrature and the
              dense per-element operators B, D_j, B^Gamma of Sec. 3.1
              (Eq. 9-10, Eq. 13)
  physics.py  conserved variables and fluxes F_i, G_i (Eq. 1-6), the Roe
              and Lax-Friedrichs Riemann fluxes, the interior-penalty face
              fluxes (Eq. 11-13)
  dg.py       residual R(u) = M^-1 L(u) (Eq. 13) written out with dense
              matrices, the stage residual N(u) (Eq. 20), L2 projection
  solver.py   Jacobian-free matvec (Eq. 25-26), block-relaxed-Jacobi
              preconditioner build and apply (Eq. 27-31), restarted
              right-preconditioned GMRES (Eq. 24), Newton (Eq. 21-23),
              SDIRK steps (Eq. 17-20, Appendix A)
  butcher.py  Butcher tableaus of Appendix A

Every function is dense and unfused; no blocking or reordering beyond what
the paper's definition states.  Readings of garbled or silent passages are
stated where they are used.
"""
