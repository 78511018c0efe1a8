"""MI355X (gfx950) T-REXI for the linearised shallow-water equations on the sphere.

The arithmetic lives in the HIP library ``librexi.so`` (C ABI in
``include/rexi.h``); this package is a thin ctypes binding with the same
entry points, using torch tensors for device memory and streams.
"""
from .rexi import (Plan, RexiError, RexiParams, Step, library_path, load_library, params_for, plan_for,
                   rexi_coeffs, run, solve_variants)

__all__ = ["Plan", "RexiError", "RexiParams", "Step", "library_path", "load_library", "params_for", "plan_for",
           "rexi_coeffs", "run", "solve_variants"]
