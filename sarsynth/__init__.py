"""Seeded synthetic near-field MIMO-SAR scans.

This package only *makes inputs*: array layouts, frequency sweeps, irregular
(freehand-like) trajectories, point/surface scenes and the echoes those scenes
return under the frequency-domain scattering model of Sec. II-C (the equation
for s(x_T, x_R, y_T, y_R, z_l, f) with P(f) = 1).  It holds none of the image
formation arithmetic (no compensation, no Fourier transforms, no Stolt map):
both the FP64 oracle and the GPU library consume what it produces.
"""

from .scans import (  # noqa: F401
    C0,
    ImageGrid,
    Scan,
    awr1443_layout,
    sweep,
    config1_scan,
    clustered_scan,
    config2_geometry,
    config2_scan,
    config4_scan,
    point_scan,
    depth_pair_scan,
    synth_echo_numpy,
    synth_echo_torch,
    add_noise_numpy,
)
