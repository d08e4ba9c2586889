"""CPU oracle for the DBFFT hot path — TEST INFRASTRUCTURE, NOT THE PRODUCT.

A plain, slow, obviously-correct FP64 NumPy implementation of what the
displacement-based FFT scheme of Lucarini & Segurado ("DBFFT: A displacement
based FFT approach for non-linear homogenization of the mechanical
behavior", arXiv:1905.12725) computes:

  * spectral.py  — frequency vectors (Sec. 2.1), the Fourier symmetric
                   gradient, full gradient and divergence operators
                   (Sec. 2.2, eqs. symgrad and diver; Sec. 2.4, eq. for g),
                   normalized transforms, the real inner product on the
                   half spectrum;
  * materials.py — linear elastic stiffness tensors, a rate-dependent J2
                   return map and a compressible neo-Hookean law (material
                   models of the workloads; not in the paper);
  * solver.py    — the linear system of eq. lineqf (strain control) and of
                   Sec. 2.3 (stress / mixed control), the preconditioner of
                   eqs. pred2/pred3, complex CG (Sec. 3 intro), the residual
                   checks of eqs. chedckeq/chedckimp, the Newton scheme of
                   Sec. 2.4 (eqs. lineariz, nonlineqf, nonlineqfstress), and
                   the adjoint gradient of a homogenized response;
  * dense.py     — an FFT-free definition of the same discrete problem
                   assembled from spectral differentiation matrices, solved
                   directly (pins the iterative route on small grids).

Only the tests, the package's smoke() and the benchmark's CPU-baseline leg
may import this package.  It shares no code with the HIP path; the two meet
only through the seeded input generators in
paper_1905_12725_amd/microstructure.py, which hold none of the method.
"""
