"""CPU oracle for mixed-precision iterative refinement on LSE / GLS problems.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything under this package: only the test-suite, the smoke check of
the entry module and the CPU-baseline leg of the benchmark use it.  It shares
no code with the HIP path.

Modules
-------
direct   FP64 reference solutions: the null-space method via the generalized RQ
         factorization for LSE and Paige's method via the generalized QR
         factorization for GLS (Section 2), augmented residuals, the stopping
         test quantities (eqs. lse-stop / gls-stop) and the accuracy metrics of
         Tables 4-5.
mpir     The paper's method itself on the CPU: Algorithms 1-4 (classical
         iterative refinement with the correction solvers) and GMRES-based
         refinement with the block-diagonal split preconditioners of
         Section 5, using LAPACK single precision for the low-precision
         factorization.
complex_lsq
         The complex problems of Section 1 (Hermitian transposes): null-space
         and Paige solutions over C, augmented residuals, stop-test scales,
         backward errors and condition numbers, with no real embedding.
extended The residual blocks computed exactly (rational arithmetic) and rounded
         once, and solutions of the augmented systems in mpmath: references
         for the extra-precise (double-double) residual.
"""
from . import complex_lsq, direct, extended, mpir  # noqa: F401
