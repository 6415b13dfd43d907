"""MI355X-native near-field MIMO-SAR image formation for irregular scanning
geometries (Smith & Torlak, IEEE Access 2022).

The compute path is the HIP library libsar.so (C ABI in include/sar.h); the
Python module `sar` is a thin ctypes binding over it.
"""

__all__ = ["sar"]
