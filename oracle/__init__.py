"""CPU FP64 oracle for the WMG-preconditioned Krylov CT reconstruction path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product library
never calls it, and it shares no code with the HIP path.

Everything here is plain and slow on purpose: the projection matrix is
assembled explicitly (scipy CSR, float64), the Haar operators are the sparse
Kronecker products that define them, and the solvers follow the paper's
recursions step by step in float64.

Modules
  geometry   - image/detector/angle conventions (Section 2.1, eq. sys)
  projector  - exact ray-pixel intersection matrix W by grid-crossing traversal
  haar       - 1D/2D Haar intergrid operators and the full packet transform
               (eq. intops, eq. intops_wav, eq. 1of4-4of4, Section 3.1.3)
  wmg        - packet diagonal, additive WMG preconditioners, Galerkin blocks
               (eq. galerkin, Section 3.1.2-3.1.3)
  solvers    - PCGLS, right-preconditioned GMRES(restart), SIRT
               (Section 2.2, eq. sirt_it, eq. kryl_sys, eq. sys_prec)

Parity status per function is listed in each module header.
"""
from . import geometry, projector, haar, wmg, solvers  # noqa: F401
