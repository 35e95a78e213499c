"""Plain CPU reference (the oracle) for classic CG and deep pipelined p(l)-CG.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import anything from this package; the
library and its Python binding never do, and nothing here calls them.

Everything is written for clarity, not speed: numpy vector operations, Python
dictionaries keyed by the paper's indices, float64 by default.  The functions
also run on numpy object arrays of ``mpmath.mpf`` values, which the tests use
to check the algebra at 50 significant digits.

Modules:
  operators - 2D 5-point / 3D 7-point Dirichlet Laplacians, dense operators,
              closed-form spectra (textbook facts used by the pins).
  shifts    - Chebyshev shifts, Eq. (chebyshev) of Sec. 2.2.
  cg        - classic Hestenes-Stiefel CG, the method p(l)-CG is compared with.
  plcg      - Alg. 1 with both dot-product forms, M = I by default or a
              given M^{-1}, the explicit restart on square-root breakdown,
              diagnostics.
  refine    - FP32-stored p(l)-CG inside FP64 iterative refinement.
"""
from . import operators, shifts, cg, plcg, refine  # noqa: F401
