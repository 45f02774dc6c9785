"""CPU oracle of the Cole-Hopf fourth-order MRT-LB scheme.

TEST INFRASTRUCTURE ONLY: the direct solver (``oracle.oracle``, C with
OpenMP) and the exact Fourier-mode evaluator (``oracle.spectral``, numpy in
extended precision).  Neither shares code with, nor imports, the HIP library.
"""
