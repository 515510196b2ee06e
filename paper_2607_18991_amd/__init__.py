"""MI355X-native Newman-Ziff first-spanning sweep for site percolation on sc(5)
with complex neighbourhoods (HIP kernels for gfx950 behind the C ABI of
include/nz.h; this package is the thin Python binding)."""
from . import nz  # noqa: F401

__all__ = ["nz"]
