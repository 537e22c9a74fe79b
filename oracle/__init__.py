"""CPU FP64 oracle for the NUFFT nonlocal-potential method (test infrastructure only).

This package is a plain, slow, obviously correct reference for what the GPU path
computes.  Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
may import it; the product library never calls into it and shares no code with it.

Modules
-------
quadrature    Fourier-space quadrature nodes and weights (Sec. 2.1, Eq. 'ifft').
potential     Direct nonuniform DFT sums for the potential (Sec. 2.1, Sec. 2.2, Alg. 1).
closed_forms  Analytic potentials of Gaussian densities used as pins (Examples 2.1-2.3).
solvers       Normalized gradient flow (Sec. 3.1) and time splitting (Sec. 4.1) on tiny grids.

Every floating-point computation is IEEE FP64, no fast-math, no reordering beyond
what a BLAS matrix product does inside one sum.
"""
from . import quadrature, potential, closed_forms, solvers  # noqa: F401
