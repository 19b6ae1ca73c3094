"""Plain FP64 CPU oracle for the neural-operator-preconditioned Helmholtz solver.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call, link or
execute this package: only the tests, the smoke check and the benchmark's CPU
baseline leg use it. It shares no code with the HIP library; the only common
dependency is the seeded input generator module ``synth``.

Modules:
  helmholtz -- the discrete operator A = Laplacian + k^2 with PML, its adjoint, dense assembly
  spectral  -- the Fourier-differentiation form of the same operator (the paper's discretization)
  unet      -- the U-Net neural operator, its reverse mode and the physics-informed loss
  fgmres    -- flexible GMRES with MGS Arnoldi and Givens least squares
  adam      -- the Adam update
"""
