"""FP64 CPU oracle for the multigrid-preconditioned Helmholtz solves of
Hong, Pham, Treister and Unser, "Diffraction Tomography with Helmholtz
Equation: Efficient and Robust Multigrid-Based Solver" (arXiv 2107.03679).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may import it.  The product (the HIP
library and its Python binding) never calls into it and shares no code with
it: the oracle assembles explicit sparse matrices (scipy.sparse, complex128)
and applies them with library products, while the HIP path is matrix-free.

Modules
  discretization  grid, absorbing layer, coefficient, assembled A (Sec. IV-A)
  multigrid       restriction/prolongation, coarse operators, damped Jacobi,
                  two-grid and multigrid cycles (Sec. III, Alg. 1-2, Sec. IV-C)
  krylov          FGMRES(m) (right preconditioned) and Bi-CGSTAB (Alg. 3)
  model           plane waves, right-hand sides, exact solves, adjoint,
                  Jacobian (Prop. 1), data fidelity, smoothed TV, gradients
  lfa             local-Fourier-analysis symbols of Sec. IV-B
  cylinder        analytic field of a dielectric cylinder (Sec. VI-A pin)
  learned         FP64 reference of the 2D learned-preconditioner network
  learned3d       FP64 reference of the 3D (3x3x3) learned-preconditioner network

Readings of passages where the paper is silent or inconsistent are listed in
the module that applies them; the product implements the same readings
independently.
"""
