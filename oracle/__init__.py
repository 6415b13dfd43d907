"""FP64 CPU oracle for near-field multi-planar MIMO-SAR image formation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test suite, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the GPU library and is written
from the paper (Smith & Torlak, "Efficient 3-D Near-Field MIMO-SAR Imaging for
Irregular Scanning Geometries"), in plain NumPy float64:

* geometry.py  exact Tx/Rx ranges (Sec. II-B, Eq. (2)), the virtual-element
  mapping (Eqs. (3)-(4)), the quadratic range expansion (Eq. (5)) and the
  residual path beta of the multi-planar compensation (Eqs. (7), (11)-(12));
* rma.py       the range-migration image formation of Sec. III, Eq. (16),
  evaluated by its plain definitions: direct 2-D non-uniform DFT, the k_z
  filter of Eq. (15), the Stolt map + z transform as a direct non-uniform sum
  over frequency, and an exact inverse DFT on the uniform (k_x, k_y) grid;
  also the same image with a reference depth per depth slab;
* bpa.py       direct back-projection with exact ranges (the gold standard the
  paper compares against, Sec. III / Sec. V).

Equation numbers count the paper's displayed equations in order
((1) far-field criterion ... (17) spatial resolution).  Every function is
pinned by tests under tests/ (printed constants, closed forms, library special
cases, invariants, brute force); see each function's docstring.
"""

from .geometry import (  # noqa: F401
    C0,
    wavenumber,
    tx_rx_coordinates,
    round_trip_exact,
    virtual_samples,
    residual_path,
    round_trip_quadratic,
    amplitude_factor,
)
from .rma import (  # noqa: F401
    mode_axes,
    compensate,
    nudft2,
    nudft2_entries,
    axial_wavenumber,
    rma_filter,
    stolt_direct,
    idft2,
    spectrum_direct,
    image_from_spectrum,
    image_planes_from_spectrum,
    reconstruct_direct,
    slab_grids,
    reconstruct_slabs,
)
from .bpa import bpa  # noqa: F401
