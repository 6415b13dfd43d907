"""Range-migration image formation of Sec. III by its plain definitions.

Test infrastructure only (see the package docstring).

The method (Eq. (16)) is

    o = IFT_3D[ S[ FT_2D[ s_hat ] * k_z / P(f) * exp(-j k_z Z_0) ] ]

with s_hat the compensated virtual planar monostatic data (Eq. (11)).  The
fast method grids the irregular (x', y') samples with a NUFFT and interpolates
onto uniform k_z (Stolt); both approximate exact sums that this module
evaluates directly:

  1. S(p, q, f_i) = sum_n s_hat_n(f_i) exp(-j [k_x,p (x'_n - x_c) + k_y,q (y'_n - y_c)])
     (forward transform, sign -j since the data carry exp(+j k_x x') in
     Eq. (13)); modes k_x,p = 2 pi p / (N_x dx), p = -N_x//2 .. N_x - N_x//2 - 1,
     centred at x_c = x0 + (N_x//2) dx (likewise in y);
  2. k_z^2 = 4 k_i^2 - k_x^2 - k_y^2 (Eq. (14)); evanescent entries
     (k_z^2 <= 0) are dropped; F = S k_z exp(-j k_z Z_0) with P(f) = 1
     (Eq. (15));
  3. Z(p, q, z_w) = sum_i F(p, q, i) exp(+j k_z,pqi z_w), z_w = z0 + w dz:
     the Stolt map followed by the z part of the inverse 3-D transform,
     written as the exact non-uniform sum it approximates; with step 2 the
     total z phase is exp(j k_z (z_w - Z_0)), the plane-wave expansion of
     Eq. (13) about the projection plane;
  4. o(x_u, y_v, z_w) = sum_{p,q} Z(p, q, z_w) exp(+j [k_x,p (x_u - x_c) + k_y,q (y_v - y_c)]),
     an exact inverse DFT on the uniform grid, unnormalised.

Array layouts: spectrum [N_y, N_x, N_f] with centred mode index
(j = p + N_x//2); image [N_x, N_y, N_z].
"""

import types

import numpy as np

from .geometry import amplitude_factor, residual_path, virtual_samples, wavenumber


def mode_axes(nx, ny, x0, y0, dx, dy):
    """Spatial-frequency axes and the lateral centre of the image grid."""
    p = np.arange(nx) - nx // 2
    q = np.arange(ny) - ny // 2
    kx = 2.0 * np.pi * p / (nx * dx)
    ky = 2.0 * np.pi * q / (ny * dy)
    return kx, ky, x0 + (nx // 2) * dx, y0 + (ny // 2) * dy


def compensate(echo, k, beta, amp=None):
    """Multi-planar multistatic compensation, Eq. (11): s_hat = s exp(+j k beta).

    echo [..., N_f], k [N_f], beta [...].  The paper's compensation is phase
    only; amp [...] (optional, amplitude_factor) also scales each sample by
    the amplitude ratio between Eqs. (9) and (10)."""
    out = np.asarray(echo, np.complex128) * np.exp(1j * np.asarray(beta)[..., None] * np.asarray(k)[None, :])
    if amp is not None:
        out = out * np.asarray(amp, np.float64)[..., None]
    return out


def nudft2(shat, xv, yv, kx, ky, xc, yc, block=8192):
    """Direct 2-D non-uniform DFT of step 1 (the FT_2D of Eq. (16)).

    shat [N_v, N_f]; xv, yv [N_v].  Evaluated per frequency as
    S_i = E_y^T diag(shat_i) E_x with E_x[n, p] = exp(-j k_x,p (x'_n - x_c)),
    accumulated over blocks of samples.  Returns [N_y, N_x, N_f]."""
    shat = np.asarray(shat, np.complex128)
    nv, nf = shat.shape
    out = np.zeros((len(ky), len(kx), nf), np.complex128)
    for b0 in range(0, nv, block):
        sl = slice(b0, b0 + block)
        ex = np.exp(-1j * np.outer(np.asarray(xv[sl]) - xc, kx))      # [b, N_x]
        ey = np.exp(-1j * np.outer(np.asarray(yv[sl]) - yc, ky))      # [b, N_y]
        for i in range(nf):
            out[:, :, i] += ey.T @ (shat[sl, i, None] * ex)
    return out


def nudft2_entries(shat, xv, yv, kx_e, ky_e, i_e, xc, yc, chunk=8):
    """Step 1 evaluated only at chosen entries (k_x,e, k_y,e, f_{i_e})."""
    shat = np.asarray(shat, np.complex128)
    xr = np.asarray(xv) - xc
    yr = np.asarray(yv) - yc
    out = np.zeros(len(kx_e), np.complex128)
    for e0 in range(0, len(kx_e), chunk):
        e = slice(e0, e0 + chunk)
        ph = np.exp(-1j * (np.outer(kx_e[e], xr) + np.outer(ky_e[e], yr)))   # [E, N_v]
        out[e] = np.einsum('en,ne->e', ph, shat[:, np.asarray(i_e[e])])
    return out


def axial_wavenumber(k, kx, ky):
    """k_z of Eq. (14) on the (k_y, k_x, k) grid: [N_y, N_x, N_f] and the
    propagating mask (k_z^2 > 0)."""
    kz2 = 4.0 * np.asarray(k)[None, None, :] ** 2 - np.asarray(kx)[None, :, None] ** 2 \
        - np.asarray(ky)[:, None, None] ** 2
    mask = kz2 > 0.0
    return np.sqrt(np.where(mask, kz2, 0.0)), mask


def rma_filter(spec, kz, mask, z_ref, k=None, dcf=False):
    """F = S k_z exp(-j k_z Z_0) / P(f), P = 1 (Eq. (15)); evanescent -> 0.

    dcf=True (the optional Jacobian of the change of variables from k to k_z,
    on which the paper is silent): F is further multiplied by
    dk_z/dk = 4 k / k_z, which follows from differentiating Eq. (14) at fixed
    (k_x, k_y); k [N_f] is then required."""
    if not dcf:
        return np.where(mask, spec * kz * np.exp(-1j * kz * float(z_ref)), 0.0)
    jac = np.where(mask, 4.0 * np.asarray(k)[None, None, :] / np.where(mask, kz, 1.0), 0.0)
    return np.where(mask, spec * kz * jac * np.exp(-1j * kz * float(z_ref)), 0.0)


def stolt_direct(filt, kz, mask, zw):
    """Step 3: Z[..., w] = sum_i F[..., i] exp(+j k_z[..., i] z_w) as an exact
    non-uniform sum (the Stolt map S plus the z transform of Eq. (16))."""
    zw = np.asarray(zw, np.float64)
    out = np.zeros(filt.shape[:-1] + (len(zw),), np.complex128)
    f = np.where(mask, filt, 0.0)
    for w, z in enumerate(zw):
        out[..., w] = np.sum(f * np.exp(1j * kz * z), axis=-1)
    return out


def idft2(zcube):
    """Step 4: o[u, v, w] = sum_{p,q} Z[q, p, w] exp(+j 2 pi (p (u - N_x//2)/N_x + q (v - N_y//2)/N_y)).

    Evaluated with the library FFT on the uniform grid: shift centred modes
    to natural order, unnormalised inverse DFT, shift the output back.
    Input [N_y, N_x, N_z], output [N_x, N_y, N_z]."""
    ny, nx = zcube.shape[0], zcube.shape[1]
    zn = np.fft.ifftshift(zcube, axes=(0, 1))
    a = np.fft.ifft2(zn, axes=(0, 1)) * (nx * ny)
    return np.ascontiguousarray(np.fft.fftshift(a, axes=(0, 1)).transpose(1, 0, 2))


def _virtual(pos, tx_xy, rx_xy, grid, compensation=True):
    xv, yv, dx, dy, dz = virtual_samples(pos, tx_xy, rx_xy, grid.z_ref)
    if compensation:
        beta = residual_path(dx, dy, dz, grid.z_ref, grid.z_focus)
    else:
        beta = np.zeros_like(xv)
    return xv.ravel(), yv.ravel(), beta.ravel()


def spectrum_direct(pos, tx_xy, rx_xy, freq, echo, grid, compensation=True, amplitude=False):
    """Compensated spatial spectrum S [N_y, N_x, N_f] (Eqs. (3)-(4), (11)-(12),
    step 1); amplitude: also apply the amplitude half (amplitude_factor at the
    grid's reference depth z_focus)."""
    k = wavenumber(freq)
    xv, yv, beta = _virtual(pos, tx_xy, rx_xy, grid, compensation)
    nf = len(k)
    amp = amplitude_factor(pos, tx_xy, rx_xy, grid.z_ref, grid.z_focus).ravel() if amplitude else None
    shat = compensate(np.asarray(echo).reshape(-1, nf), k, beta, amp)
    kx, ky, xc, yc = mode_axes(grid.nx, grid.ny, grid.x0, grid.y0, grid.dx, grid.dy)
    return nudft2(shat, xv, yv, kx, ky, xc, yc)


def image_from_spectrum(spec, freq, grid, dcf=False):
    """Steps 2-4 on a spectrum [N_y, N_x, N_f]; returns the image [N_x, N_y, N_z]
    (dcf: see rma_filter)."""
    k = wavenumber(freq)
    kx, ky, _, _ = mode_axes(grid.nx, grid.ny, grid.x0, grid.y0, grid.dx, grid.dy)
    kz, mask = axial_wavenumber(k, kx, ky)
    filt = rma_filter(spec, kz, mask, grid.z_ref, k, dcf)
    zw = grid.z0 + grid.dz * np.arange(grid.nz)
    return idft2(stolt_direct(filt, kz, mask, zw))


def image_planes_from_spectrum(spec, freq, grid, w_list, row_chunk=16, dcf=False):
    """Steps 2-4 for selected z planes only; returns [N_x, N_y, len(w_list)].
    Chunked over k_y rows so large spectra fit in memory."""
    k = wavenumber(freq)
    kx, ky, _, _ = mode_axes(grid.nx, grid.ny, grid.x0, grid.y0, grid.dx, grid.dy)
    zw = grid.z0 + grid.dz * np.asarray(w_list, np.float64)
    zc = np.zeros((grid.ny, grid.nx, len(zw)), np.complex128)
    for r0 in range(0, grid.ny, row_chunk):
        rs = slice(r0, r0 + row_chunk)
        kz, mask = axial_wavenumber(k, kx, ky[rs])
        filt = rma_filter(np.asarray(spec[rs], np.complex128), kz, mask, grid.z_ref, k, dcf)
        zc[rs] = stolt_direct(filt, kz, mask, zw)
    return idft2(zc)


def reconstruct_direct(pos, tx_xy, rx_xy, freq, echo, grid, compensation=True, dcf=False, amplitude=False):
    """Full image [N_x, N_y, N_z] of one scan (Fig. 3 pipeline, Eq. (16));
    dcf: see rma_filter; amplitude: see spectrum_direct."""
    spec = spectrum_direct(pos, tx_xy, rx_xy, freq, echo, grid, compensation, amplitude)
    return image_from_spectrum(spec, freq, grid, dcf)


def slab_grids(grid, n_slabs):
    """Depth slabs of an image grid: slab j holds planes [j n, (j + 1) n),
    n = N_z / n_slabs, with its reference depth z_c,j at the z-centre of those
    planes.  The residual path of Eqs. (7), (12) then uses R_c,j = |z_c,j - Z_0|
    for the targets of slab j (the paper attributes its depth aberrations to a
    single reference depth, Sec. V-A)."""
    if n_slabs < 1 or grid.nz % n_slabs:
        raise ValueError("n_slabs must divide N_z")
    n = grid.nz // n_slabs
    out = []
    for j in range(n_slabs):
        z0 = grid.z0 + j * n * grid.dz
        out.append(types.SimpleNamespace(nx=grid.nx, ny=grid.ny, nz=n, x0=grid.x0, y0=grid.y0, z0=z0,
                                         dx=grid.dx, dy=grid.dy, dz=grid.dz, z_ref=grid.z_ref,
                                         z_focus=z0 + 0.5 * (n - 1) * grid.dz))
    return out


def reconstruct_slabs(pos, tx_xy, rx_xy, freq, echo, grid, n_slabs, amplitude=False):
    """Image [N_x, N_y, N_z] with a reference depth per depth slab: slab j is
    the direct reconstruction of Eq. (16) on the slab's planes, compensated with
    the slab's own reference depth (slab_grids), in phase and, with amplitude,
    in amplitude."""
    img = np.zeros((grid.nx, grid.ny, grid.nz), np.complex128)
    for j, g in enumerate(slab_grids(grid, n_slabs)):
        img[:, :, j * g.nz:(j + 1) * g.nz] = reconstruct_direct(pos, tx_xy, rx_xy, freq, echo, g,
                                                                amplitude=amplitude)
    return img
