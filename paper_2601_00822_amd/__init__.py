"""MI355X-native BFCS Lippmann-Schwinger FFT solver (liblsfft) and its binding.

The solver is the HIP library ``liblsfft.so`` built from ``csrc/`` for gfx950
(C ABI in ``include/lsfft.h``); ``lsfft`` is its ctypes binding.
"""
from .lsfft import (Plan, LsfftError, SolveReport, lame_from_young, load_library, status_string,  # noqa: F401
                    block_mean, sample_norms, relative_l2, bump_forces, nonlocal_normal_equations,
                    nonlocal_apply, nonlocal_fit,
                    OK, W_STAGNATED, E_ARG, E_ALLOC, E_DEVICE, E_NOCONV, E_NONEQUIL, E_DIVERGED,
                    K_XPASS, K_YPASS, K_GREEN, K_REDUCE, K_CGUPD, K_OTHER)
