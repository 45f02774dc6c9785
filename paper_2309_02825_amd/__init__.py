"""MI355X (gfx950) implementation of the Cole-Hopf fourth-order MRT lattice
Boltzmann solver for the d-dimensional coupled Burgers equations
(Chen, Liu, Chai & Shi, arXiv:2309.02825).

Modules
  lbm        ctypes binding of the C ABI in include/lbm.h (liblbm_hip.so)
  solver     Solver / BatchSolver / differentiable velocity() over that ABI
  workloads  seeded synthetic inputs and closed-form heat-equation solutions
  build      compiles the HIP library for gfx950

Importing the package loads nothing; the HIP library is loaded on first use
and its absence is an error (there is no fallback path).
"""
