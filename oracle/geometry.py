"""Geometry of the multi-planar multistatic aperture (Sec. II-B).

Test infrastructure only (see the package docstring).
"""

import numpy as np

C0 = 299_792_458.0  # speed of light (m/s); with it c / 79 GHz = 3.79 mm as printed in Sec. V-A


def wavenumber(freq_hz):
    """k = 2 pi f / c, the instantaneous wavenumber of Sec. II-C (Eq. (9))."""
    return 2.0 * np.pi * np.asarray(freq_hz, np.float64) / C0


def tx_rx_coordinates(pos, tx_xy, rx_xy):
    """Absolute Tx and Rx coordinates of every (shot, Tx, Rx) triple.

    pos [N_pos, 3] is the device origin per shot; tx_xy [n_tx, 2] and
    rx_xy [n_rx, 2] are in-plane offsets, so Tx and Rx of one shot share the
    shot's z, i.e. they lie on the same plane z_l (Sec. II-B).
    Returns xT, yT, xR, yR, zl, each [N_pos, n_tx * n_rx] (pair = t*n_rx + r).
    """
    pos = np.asarray(pos, np.float64)
    n_tx, n_rx = len(tx_xy), len(rx_xy)
    t = np.repeat(np.arange(n_tx), n_rx)
    r = np.tile(np.arange(n_rx), n_tx)
    xT = pos[:, 0, None] + np.asarray(tx_xy, np.float64)[t, 0][None, :]
    yT = pos[:, 1, None] + np.asarray(tx_xy, np.float64)[t, 1][None, :]
    xR = pos[:, 0, None] + np.asarray(rx_xy, np.float64)[r, 0][None, :]
    yR = pos[:, 1, None] + np.asarray(rx_xy, np.float64)[r, 1][None, :]
    zl = np.broadcast_to(pos[:, 2, None], xT.shape).copy()
    return xT, yT, xR, yR, zl


def round_trip_exact(xT, yT, xR, yR, zl, point):
    """R^RT = R^T + R^R between the pair and a point scatterer (Eq. (2))."""
    x, y, z = (float(v) for v in point)
    rt = np.sqrt((xT - x) ** 2 + (yT - y) ** 2 + (zl - z) ** 2)
    rr = np.sqrt((xR - x) ** 2 + (yR - y) ** 2 + (zl - z) ** 2)
    return rt + rr


def virtual_samples(pos, tx_xy, rx_xy, z_ref):
    """Virtual planar monostatic element of every Tx/Rx pair and shot.

    Inverting Eq. (3): x' = (x_T + x_R)/2, d^x = x_R - x_T (same in y), and
    Eq. (4): d^z = z_l - Z_0.  Returns (xv, yv, dx, dy, dz), each
    [N_pos, n_tx * n_rx].
    """
    xT, yT, xR, yR, zl = tx_rx_coordinates(pos, tx_xy, rx_xy)
    xv = 0.5 * (xT + xR)
    yv = 0.5 * (yT + yR)
    return xv, yv, xR - xT, yR - yT, zl - float(z_ref)


def residual_path(dx, dy, dz, z_ref, z_focus):
    """Residual path beta of the multi-planar compensation (Eqs. (7), (12)).

    The paper derives beta = 2 d^z + (d_x^2 + d_y^2) / (4 Z_0) after moving the
    target to the origin, so there "Z_0" is the array-to-scene distance and the
    array sits on the +z side of the scene.  In a frame with the projection
    plane at z = Z_0 and a scene reference depth z_c, the first-order term of
    Eq. (5) is 2 (Z_0 - z) d^z / R_0 ~ 2 sign(Z_0 - z_c) d^z and the
    multistatic term's denominator is R_c = |z_c - Z_0|:

        beta = 2 sign(Z_0 - z_c) d^z + (d_x^2 + d_y^2) / (4 R_c).
    """
    rc = abs(float(z_focus) - float(z_ref))
    if rc <= 0.0:
        raise ValueError("scene reference depth must differ from the projection plane")
    s = np.sign(float(z_ref) - float(z_focus))
    return 2.0 * s * np.asarray(dz) + (np.asarray(dx) ** 2 + np.asarray(dy) ** 2) / (4.0 * rc)


def round_trip_quadratic(xv, yv, dx, dy, dz, z_ref, point):
    """Second-order expansion of R^RT in (d^x, d^y, d^z) about the virtual
    element (Eq. (5); derived in the Appendix)."""
    x, y, z = (float(v) for v in point)
    z0 = float(z_ref)
    r0 = np.sqrt((xv - x) ** 2 + (yv - y) ** 2 + (z0 - z) ** 2)     # Eq. (6)
    return (2.0 * r0 + 2.0 * (z0 - z) * dz / r0
            + (dx ** 2 + dy ** 2 + 4.0 * dz ** 2) / (4.0 * r0)
            - (((xv - x) * dx + (yv - y) * dy) ** 2 + 4.0 * (z0 - z) ** 2 * dz ** 2) / (4.0 * r0 ** 3))


def amplitude_factor(pos, tx_xy, rx_xy, z_ref, z_focus):
    """Amplitude half of the compensation: the ratio R^T R^R / R_0^2 that turns
    the multistatic amplitude 1/(R^T R^R) of Eq. (9) into the planar monostatic
    amplitude 1/R_0^2 of Eq. (10), evaluated for a reference scatterer straight
    ahead of each virtual element, at (x', y', z_c) with z_c the scene (or
    slab) reference depth.  R^T and R^R are the exact ranges of Eq. (2) from
    the pair's Tx and Rx, R_0 the range of Eq. (6) from the virtual element on
    the plane Z_0.  Returns [N_pos, n_tx * n_rx]; 1 for a monostatic element
    on the plane."""
    xT, yT, xR, yR, zl = tx_rx_coordinates(pos, tx_xy, rx_xy)
    xv, yv = 0.5 * (xT + xR), 0.5 * (yT + yR)
    zc = float(z_focus)
    rt = np.sqrt((xT - xv) ** 2 + (yT - yv) ** 2 + (zl - zc) ** 2)
    rr = np.sqrt((xR - xv) ** 2 + (yR - yv) ** 2 + (zl - zc) ** 2)
    r0 = abs(zc - float(z_ref))
    if r0 <= 0.0:
        raise ValueError("scene reference depth must differ from the projection plane")
    return rt * rr / r0 ** 2
