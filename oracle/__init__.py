"""FP64 CPU oracle for the fast-LGF Navier-Stokes hot path.  TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check of the package entry file and the CPU-baseline leg of the
benchmark may import, call, link or run anything in this package.  The product path (the HIP
library and its Python binding) never routes through it and shares no code with it.

Each function is a plain, slow, obviously correct restatement of the paper
(Liska & Colonius, "A fast lattice Green's function method for solving viscous incompressible
flows on unbounded domains"):

* ``lgf``      -- lattice Green's function of the 7-point Laplacian from its Bessel-integral form
                  (Appendix B), by adaptive quadrature over library Bessel functions.
* ``native``   -- direct O(N_src * N_tgt) lattice summation of the LGF convolution
                  (Sec. 2.2, Eq. dpoisson_conv), plain C with compensated accumulation.
* ``stencils`` -- the point operators of Appendix A (G, Dbar, C, Cbar, D, Gbar, L, Ntilde),
                  zero outside the box (mask operators, Sec. 4.1).
* ``intfac``   -- integrating-factor kernel e^{-2a} I_k(2a) per axis (Appendix B, Eq. lgf_intfac)
                  applied as an unseparated 3D sum (Sec. 2.3, Eq. if_def).
* ``ifherk``   -- the IF-HERK step in its plain (non-shortcut) recursion (Sec. 3.2) with the
                  projection of Sec. 3.3 and the masked form of Sec. 5, plus Vor2Vel (Sec. 4.1).
* ``conv3d``   -- FP64 reference of the learned surrogate's layers (not part of the paper).
"""
