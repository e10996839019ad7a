"""Two-level DD-alpha-AMG for Wilson-clover fermions on one AMD gfx950 GPU.

The compute path is the HIP library libdd.so (C ABI in include/dd.h); this
package holds its sources (csrc/), the build script and a thin ctypes binding.
"""
from .binding import (Context, Gauge, MG, SolveState, DDError, default_params, bicgstab_params, level3_params, lib, load,  # noqa: F401
                      DD_F64, DD_F32, DD_F16, DD_BF16, DTYPES)
