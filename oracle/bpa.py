"""Direct back-projection with exact bistatic ranges.

Test infrastructure only (see the package docstring).

The paper's gold standard (Sec. III, Sec. V): every voxel correlates all
samples with the exact round-trip phase of Eq. (2) under the model of Eq. (9),

    o_B(r) = sum_n sum_i s_n(f_i) exp(+j k_i (R^T_n(r) + R^R_n(r))),

unit amplitude weight.  Cost N_v * N_f * N_voxels: tiny scans only.
"""

import numpy as np

from .geometry import tx_rx_coordinates, wavenumber


def bpa(pos, tx_xy, rx_xy, freq, echo, grid, voxel_chunk=512):
    k = wavenumber(freq)
    xT, yT, xR, yR, zl = (a.ravel() for a in tx_rx_coordinates(pos, tx_xy, rx_xy))
    s = np.asarray(echo, np.complex128).reshape(-1, len(k))                  # [N_v, N_f]
    xs, ys, zs = grid.coords()
    vx, vy, vz = (a.ravel() for a in np.meshgrid(xs, ys, zs, indexing='ij'))
    out = np.zeros(vx.size, np.complex128)
    for c0 in range(0, vx.size, voxel_chunk):
        c = slice(c0, c0 + voxel_chunk)
        rt = np.sqrt((xT[:, None] - vx[None, c]) ** 2 + (yT[:, None] - vy[None, c]) ** 2
                     + (zl[:, None] - vz[None, c]) ** 2)
        rr = np.sqrt((xR[:, None] - vx[None, c]) ** 2 + (yR[:, None] - vy[None, c]) ** 2
                     + (zl[:, None] - vz[None, c]) ** 2)
        r = rt + rr                                                           # [N_v, chunk]
        for i in range(len(k)):
            out[c] += s[:, i] @ np.exp(1j * k[i] * r)
    return out.reshape(grid.nx, grid.ny, grid.nz)
