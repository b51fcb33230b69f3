"""MI355X-native explicit upwind DG for velocity-strain elastic waves on tetrahedra.

The compute path is the HIP library libewdg.so (C ABI in include/ewdg.h);
this package holds its sources (csrc/), the build script and a thin ctypes
binding (ewdg.Context).
"""
from .ewdg import Context, EwdgError, Transport, batch_table_bytes, load, step_batch  # noqa: F401
