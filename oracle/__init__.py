"""FP64 CPU oracle for the BFCS modified Lippmann-Schwinger FFT method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package: only ``tests/``, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP path.

Modules:

* ``lsfft_oracle`` -- plain NumPy implementations, in float64, of the method's
  steps in the paper's order: Algorithm 1 (modified basic scheme, Sec. 5,
  Eqs. 5.7-5.11), Algorithm 2 (Krylov form, Eqs. 5.12-5.13), the
  displacement form it is equivalent to (Eqs. 5.14-5.17), the classical
  Lippmann-Schwinger mode (Eqs. 2.24, 5.1-5.2) and the translated averages of
  Sec. 3 (Eqs. 3.3-3.7).
* ``dense`` -- a brute-force dense assembly and direct solve of the same
  discrete system, built from explicit DFT matrices (no FFT library), used to
  pin the iterative oracle on tiny grids.
"""
from . import lsfft_oracle, dense  # noqa: F401
