"""Plain FP64 CPU oracle for the modal DG ideal-MHD scheme of Guillet et al.,
"High-order magnetohydrodynamics for astrophysics with an adaptive mesh
refinement discontinuous Galerkin scheme" (MNRAS 2019, arXiv:1806.02343).

TEST INFRASTRUCTURE ONLY.  This package is the independent reference against
which the HIP library is checked.  Only the tests, the smoke entry point and
the benchmark's CPU-baseline leg may import it; the product path never does.
It shares no code with the HIP library (its own quadrature, bases, Riemann
solver, limiters, eigen-systems and mesh logic) and is written for clarity,
not speed: numpy arrays vectorised over cells / faces / points, FP64
throughout, no blocking or fusion beyond what the paper's formulas state.

Modules
  quadrature  Gauss-Legendre rules (Sec. 3.5)
  basis       Legendre and locally divergence-free bases (Sec. 3.2-3.3, App. A)
  physics     EOS, ideal-MHD flux, HLLD, face B_n choice, GLM upwinding,
              Powell q (Sec. 2, Sec. 4.1)
  dg          weak-form right-hand side, time step, SSP-RK3 (Sec. 3.5-3.6, 4.1)
  limiters    TVB characteristic slope limiter, LDF slope fix, positivity
              limiter (Sec. 4.2-4.3)
  eigen       1-D MHD characteristic matrices used by the slope limiter
  amr         octree mesh with 2:1 hanging faces (Sec. 4.4)
  mlp         learned troubled-cell indicator (forward/backward, FP64/FP32)
"""
