"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test ties one oracle function to something other than itself: numbers
printed in the paper (tests/golden), closed forms the paper derives (the
Appendix derivatives, Eq. (17) resolution), library special cases (FFT),
invariants (Parseval, shift, rigid z-translation, linearity) and brute force
on tiny inputs, chosen so that a dropped term, a wrong sign, a wrong index or
a transposed operand fails at least one of them.
"""

import dataclasses
import json
import os

import numpy as np
import pytest

import oracle
from oracle import geometry as geo
from oracle import rma
from sarsynth import ImageGrid, awr1443_layout, depth_pair_scan, point_scan, synth_echo_numpy, sweep

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


# --------------------------------------------------------------------------
# printed constants (Sec. III, Sec. IV, Sec. V-A)
# --------------------------------------------------------------------------

def test_printed_constants():
    g = _gold("paper_constants.json")
    lam = oracle.C0 / g["center_wavelength"]["freq_hz"]
    assert round(lam * 1e3, 2) == g["center_wavelength"]["lambda_mm"]
    d = g["dz_max_vs_wavelength"]
    assert d["dz_max_m"] / lam > d["more_than_wavelengths"]
    p = g["prf_lower_bound"]
    prf_khz = 4.0 * p["v_max_mps"] / (oracle.C0 / p["freq_hz"]) / 1e3
    assert abs(prf_khz - p["prf_khz_approx"]) < p["approx_tol_khz"]
    k = oracle.wavenumber([g["center_wavelength"]["freq_hz"]])[0]
    assert abs(k - 2 * np.pi / lam) < 1e-9 * k


# --------------------------------------------------------------------------
# virtual elements (Eqs. (3)-(4))
# --------------------------------------------------------------------------

def test_awr1443_virtual_array():
    g = _gold("awr1443_virtual_array.json")
    lam = oracle.C0 / 79e9
    tx = np.array([[0.0, y * lam] for y in g["tx_y"]])
    rx = np.array([[0.0, y * lam] for y in g["rx_y"]])
    xv, yv, dx, dy, dz = oracle.virtual_samples(np.zeros((1, 3)), tx, rx, z_ref=0.0)
    np.testing.assert_allclose(yv[0] / lam, g["virtual_y"], atol=1e-12)
    np.testing.assert_allclose(dy[0] / lam, g["separation_y"], atol=1e-12)
    assert np.all(xv == 0) and np.all(dx == 0) and np.all(dz == 0)
    # the sarsynth layout is the same array
    tx2, rx2 = awr1443_layout()
    np.testing.assert_allclose(tx2 / lam, tx / lam, atol=1e-12)
    np.testing.assert_allclose(rx2 / lam, rx / lam, atol=1e-12)


def test_virtual_plane_offset():
    # Eq. (4): z_l = Z_0 + d^z; Eq. (3): Tx and Rx are symmetric about x'
    pos = np.array([[0.01, -0.02, 0.013]])
    tx = np.array([[0.003, -0.001]])
    rx = np.array([[-0.002, 0.004]])
    xv, yv, dx, dy, dz = oracle.virtual_samples(pos, tx, rx, z_ref=0.005)
    assert abs(dz[0, 0] - 0.008) < 1e-15
    xT, yT, xR, yR, _ = geo.tx_rx_coordinates(pos, tx, rx)
    assert abs((xv - dx / 2) - xT).max() < 1e-15 and abs((xv + dx / 2) - xR).max() < 1e-15
    assert abs((yv - dy / 2) - yT).max() < 1e-15 and abs((yv + dy / 2) - yR).max() < 1e-15


# --------------------------------------------------------------------------
# exact range vs the Appendix derivatives; residual path order and sign
# --------------------------------------------------------------------------

def _rt_of_d(xv, yv, z0, d, point):
    dxx, dyy, dzz = d
    return geo.round_trip_exact(np.array(xv - dxx / 2), np.array(yv - dyy / 2), np.array(xv + dxx / 2),
                                np.array(yv + dyy / 2), np.array(z0 + dzz), point)


@pytest.mark.parametrize("case", range(4))
def test_appendix_derivatives(case):
    rng = np.random.default_rng(100 + case)
    xv, yv, z0 = rng.uniform(-0.1, 0.1), rng.uniform(-0.1, 0.1), rng.uniform(-0.02, 0.02)
    pt = (rng.uniform(-0.1, 0.1), rng.uniform(-0.1, 0.1), rng.uniform(0.2, 0.5))
    x, y, z = pt
    r0 = np.sqrt((xv - x) ** 2 + (yv - y) ** 2 + (z0 - z) ** 2)
    f = lambda d: float(_rt_of_d(xv, yv, z0, d, pt))   # noqa: E731
    h = 1e-4
    e = np.eye(3)
    grad = np.array([(f(h * e[i]) - f(-h * e[i])) / (2 * h) for i in range(3)])
    # Appendix, first derivatives (the third is with respect to d^z)
    np.testing.assert_allclose(grad, [0.0, 0.0, 2 * (z0 - z) / r0], atol=1e-8)
    h = 4e-4
    hess = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            hess[i, j] = (f(h * e[i] + h * e[j]) - f(h * e[i] - h * e[j]) - f(-h * e[i] + h * e[j])
                          + f(-h * e[i] - h * e[j])) / (4 * h * h)
    paper = np.array([
        [(1 - (xv - x) ** 2 / r0 ** 2) / (2 * r0), -(xv - x) * (yv - y) / (2 * r0 ** 3), 0.0],
        [-(xv - x) * (yv - y) / (2 * r0 ** 3), (1 - (yv - y) ** 2 / r0 ** 2) / (2 * r0), 0.0],
        [0.0, 0.0, 2 * (1 - (z0 - z) ** 2 / r0 ** 2) / r0]])
    np.testing.assert_allclose(hess, paper, atol=2e-5 * np.abs(paper).max())


@pytest.mark.parametrize("frame", ["array_at_zero", "array_above_scene"])
def test_residual_path_is_third_order_on_axis(frame):
    # beta must absorb every first and second order term of R^RT - 2 R_0 for a
    # scatterer on the virtual element's axis at the reference depth: the
    # remainder then scales with |d|^3 (a wrong sign leaves O(d), a wrong
    # denominator O(d^2)).
    if frame == "array_at_zero":
        z_ref, z_c = 0.0, 0.3
    else:                      # the paper's own frame: scene at the origin, array at +Z_0
        z_ref, z_c = 0.3, 0.0
    xv, yv = 0.012, -0.007
    pt = (xv, yv, z_c)
    d0 = np.array([0.004, 0.006, 0.008])
    errs = []
    for s in (1.0, 0.5, 0.25):
        d = s * d0
        r0 = abs(z_c - z_ref)
        beta = oracle.residual_path(d[0], d[1], d[2], z_ref, z_c)
        errs.append(float(_rt_of_d(xv, yv, z_ref, d, pt)) - 2 * r0 - float(beta))
    errs = np.abs(errs)
    assert errs[0] < 1e-5
    assert 6.0 < errs[0] / errs[1] < 10.0 and 6.0 < errs[1] / errs[2] < 10.0


def test_residual_path_sign_reading():
    # array plane at 0, scatterer at +0.3 m: moving the device 3 mm towards the
    # scene shortens the round trip by about 6 mm (beta = -2 d^z), not +6 mm.
    pt = (0.0, 0.0, 0.3)
    for dzz in (-3e-3, 3e-3):
        exact = float(_rt_of_d(0.0, 0.0, 0.0, (0.0, 0.0, dzz), pt)) - 0.6
        beta = float(oracle.residual_path(0.0, 0.0, dzz, 0.0, 0.3))
        assert abs(exact - beta) < 5e-5
        assert abs(exact - 2 * dzz) > 1e-2


def test_quadratic_expansion_off_axis():
    # Eq. (5) keeps every second-order term for any scatterer position
    xv, yv, z0 = 0.02, -0.015, 0.0
    pt = (-0.03, 0.025, 0.27)
    d0 = np.array([0.005, -0.004, 0.01])
    errs = []
    for s in (1.0, 0.5, 0.25):
        d = s * d0
        q = oracle.round_trip_quadratic(np.array(xv), np.array(yv), d[0], d[1], d[2], z0, pt)
        errs.append(abs(float(_rt_of_d(xv, yv, z0, d, pt)) - float(q)))
    assert 6.0 < errs[0] / errs[1] < 10.0 and 6.0 < errs[1] / errs[2] < 10.0


def test_compensation_recovers_planar_model():
    # data built with the expanded range 2R_0 + beta and amplitude 1/R_0^2 must
    # compensate to the virtual planar monostatic response of Eq. (10)
    rng = np.random.default_rng(5)
    tx, rx = awr1443_layout()
    pos = np.stack([rng.uniform(-0.05, 0.05, 20), rng.uniform(-0.05, 0.05, 20), rng.uniform(-0.02, 0.02, 20)], 1)
    freq = sweep(16)
    k = oracle.wavenumber(freq)
    xv, yv, dx, dy, dz = oracle.virtual_samples(pos, tx, rx, 0.0)
    beta = oracle.residual_path(dx, dy, dz, 0.0, 0.3)
    pt = (0.01, -0.02, 0.31)
    r0 = np.sqrt((xv - pt[0]) ** 2 + (yv - pt[1]) ** 2 + pt[2] ** 2)
    s = np.exp(-1j * k * (2 * r0 + beta)[..., None]) / (r0 ** 2)[..., None]
    shat = oracle.compensate(s, k, beta)
    ref = np.exp(-2j * k * r0[..., None]) / (r0 ** 2)[..., None]
    assert np.abs(shat - ref).max() < 1e-12 * np.abs(ref).max()


def test_amplitude_factor_restores_the_planar_amplitude():
    # the amplitude half of the compensation: for a scatterer straight ahead of
    # a virtual element at the reference depth z_c, the echo of Eq. (9) (built
    # by the input generator with exact ranges and amplitude 1/(R^T R^R))
    # scaled by the factor has the planar amplitude 1/R_0^2 of Eq. (10), for
    # tilted shots (d^z != 0) and every Tx/Rx pair; without it the amplitude is
    # off by up to tens of percent
    rng = np.random.default_rng(11)
    tx = np.array([[-0.03, 0.0], [0.03, 0.01]])
    rx = np.array([[-0.01, 0.0], [0.01, -0.02], [0.0, 0.02]])
    z_ref, z_c = 0.0, 0.25
    pos = np.stack([rng.uniform(-0.05, 0.05, 6), rng.uniform(-0.05, 0.05, 6), rng.uniform(-0.03, 0.03, 6)], 1)
    freq = sweep(4)
    k = oracle.wavenumber(freq)
    xv, yv, dx, dy, dz = oracle.virtual_samples(pos, tx, rx, z_ref)
    amp = oracle.amplitude_factor(pos, tx, rx, z_ref, z_c)
    beta = oracle.residual_path(dx, dy, dz, z_ref, z_c)
    worst_without = 0.0
    for m in range(len(pos)):
        for l in range(len(tx) * len(rx)):
            tgt = np.array([[xv[m, l], yv[m, l], z_c]])
            s = synth_echo_numpy(pos[m:m + 1], tx, rx, freq, tgt, np.ones(1, np.complex128))[0, l]
            shat = oracle.compensate(s[None, :], k, beta[m, l:l + 1], amp[m, l:l + 1])[0]
            planar = 1.0 / (z_c - z_ref) ** 2
            assert np.abs(np.abs(shat) / planar - 1).max() < 1e-12
            worst_without = max(worst_without, float(np.abs(np.abs(s) / planar - 1).max()))
    assert worst_without > 0.1
    # a monostatic element on the projection plane needs no amplitude change
    on_plane = np.stack([pos[:, 0], pos[:, 1], np.full(len(pos), z_ref)], 1)
    z2 = np.zeros((1, 2))
    assert np.array_equal(oracle.amplitude_factor(on_plane, z2, z2, z_ref, z_c), np.ones((len(pos), 1)))


def test_one_slab_with_amplitude_is_the_single_depth_image_with_amplitude():
    sc = depth_pair_scan(n_side=8, n_freq=4)
    g = sc.grid
    o1 = oracle.reconstruct_slabs(sc.pos, sc.tx_xy, sc.rx_xy, sc.freq, sc.echo, g, 1, amplitude=True)
    gc = dataclasses.replace(g, z_focus=g.z0 + 0.5 * (g.nz - 1) * g.dz)
    o2 = oracle.reconstruct_direct(sc.pos, sc.tx_xy, sc.rx_xy, sc.freq, sc.echo, gc, amplitude=True)
    assert np.array_equal(o1, o2)
    o3 = oracle.reconstruct_direct(sc.pos, sc.tx_xy, sc.rx_xy, sc.freq, sc.echo, gc)
    assert _rel(o2, o3) > 1e-3


# --------------------------------------------------------------------------
# 2-D non-uniform DFT
# --------------------------------------------------------------------------

def test_nudft_on_lattice_equals_fft_and_parseval():
    rng = np.random.default_rng(7)
    nx, ny, nf = 8, 6, 3
    dx, dy = 1.3e-3, 0.9e-3
    kx, ky, xc, yc = oracle.mode_axes(nx, ny, -0.004, 0.002, dx, dy)
    a = np.arange(nx) - nx // 2
    b = np.arange(ny) - ny // 2
    bb, aa = np.meshgrid(b, a, indexing='ij')               # [ny, nx]
    xv = (xc + aa * dx).ravel()
    yv = (yc + bb * dy).ravel()
    s = rng.standard_normal((ny * nx, nf)) + 1j * rng.standard_normal((ny * nx, nf))
    spec = oracle.nudft2(s, xv, yv, kx, ky, xc, yc, block=7)
    lib = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(s.reshape(ny, nx, nf), axes=(0, 1)), axes=(0, 1)),
                          axes=(0, 1))
    assert _rel(spec, lib) < 1e-12
    assert abs(np.sum(np.abs(spec) ** 2) - nx * ny * np.sum(np.abs(s) ** 2)) < 1e-10 * np.sum(np.abs(spec) ** 2)


def test_nudft_bruteforce_tiny():
    rng = np.random.default_rng(8)
    nv, nx, ny, nf = 7, 4, 6, 3
    kx, ky, xc, yc = oracle.mode_axes(nx, ny, -0.01, -0.02, 2e-3, 3e-3)
    xv = rng.uniform(-0.02, 0.02, nv)
    yv = rng.uniform(-0.03, 0.03, nv)
    s = rng.standard_normal((nv, nf)) + 1j * rng.standard_normal((nv, nf))
    ref = np.zeros((ny, nx, nf), complex)
    for q in range(ny):
        for p in range(nx):
            for i in range(nf):
                for n in range(nv):
                    ref[q, p, i] += s[n, i] * np.exp(-1j * (kx[p] * (xv[n] - xc) + ky[q] * (yv[n] - yc)))
    assert _rel(oracle.nudft2(s, xv, yv, kx, ky, xc, yc, block=3), ref) < 1e-13
    sel = [(0, 0, 0), (3, 5, 2), (1, 2, 1)]
    ent = oracle.nudft2_entries(s, xv, yv, np.array([kx[p] for p, q, i in sel]),
                                np.array([ky[q] for p, q, i in sel]), np.array([i for p, q, i in sel]), xc, yc)
    np.testing.assert_allclose(ent, [ref[q, p, i] for p, q, i in sel], rtol=1e-13)


def test_single_sample_at_centre_is_flat():
    kx, ky, xc, yc = oracle.mode_axes(10, 8, 0.0, 0.0, 1e-3, 1e-3)
    s = np.array([[2.0 - 1.0j]])
    spec = oracle.nudft2(s, np.array([xc]), np.array([yc]), kx, ky, xc, yc)
    assert np.abs(spec - s[0, 0]).max() < 1e-15


# --------------------------------------------------------------------------
# filter, Stolt sum, inverse DFT
# --------------------------------------------------------------------------

def test_axial_wavenumber_special_cases():
    k = oracle.wavenumber(sweep(5))
    kz, mask = oracle.axial_wavenumber(k, np.array([0.0, 3 * k[-1]]), np.array([0.0]))
    np.testing.assert_allclose(kz[0, 0], 2 * k, rtol=1e-15)
    assert mask[0, 0].all() and not mask[0, 1].any() and np.all(kz[0, 1] == 0)


def test_stolt_sum_uniform_kz_is_inverse_fft():
    rng = np.random.default_rng(11)
    n, dz = 16, 2.5e-3
    f = rng.standard_normal((2, 3, n)) + 1j * rng.standard_normal((2, 3, n))
    kz = np.broadcast_to(2 * np.pi * np.arange(n) / (n * dz), f.shape)
    z = oracle.stolt_direct(f, kz, np.ones(f.shape, bool), dz * np.arange(n))
    assert _rel(z, n * np.fft.ifft(f, axis=-1)) < 1e-12


def test_stolt_jacobian_option_turns_the_sum_into_an_integral_over_kz():
    # With the optional Jacobian dk_z/dk = 4k/k_z (differentiating Eq. (14) at
    # fixed lateral wavenumber) a trapezoid-weighted sum over the frequency
    # samples of one column, sum_i w_i (dk_z/dk)_i exp(j k_z,i z), is the
    # integral over k_z of exp(j k_z z), whose closed form is
    # (exp(j k_z,hi z) - exp(j k_z,lo z)) / (j z).  The spectrum 1/k_z cancels
    # the filter's own k_z factor of Eq. (15).  Without the option (or with a
    # wrong factor) the sum is an integral over k instead and misses by about
    # the Jacobian, about 2.35 to 2.39 along this column.
    k = oracle.wavenumber(np.linspace(77e9, 81e9, 8001))
    dk = k[1] - k[0]
    kx, ky = np.array([1.1 * k[0]]), np.array([0.0])
    kz, mask = oracle.axial_wavenumber(k, kx, ky)
    assert mask.all()
    w = np.full(len(k), dk)
    w[0] = w[-1] = 0.5 * dk
    spec = (w / kz[0, 0])[None, None, :]
    z = np.array([0.05, 0.13, 0.3])
    lo, hi = kz[0, 0, 0], kz[0, 0, -1]
    ref = (np.exp(1j * hi * z) - np.exp(1j * lo * z)) / (1j * z)
    got = oracle.stolt_direct(oracle.rma_filter(spec, kz, mask, 0.0, k, dcf=True), kz, mask, z)[0, 0]
    assert _rel(got, ref) < 1e-4
    plain = oracle.stolt_direct(oracle.rma_filter(spec, kz, mask, 0.0), kz, mask, z)[0, 0]
    assert _rel(plain, ref) > 0.3


def test_idft2_bruteforce():
    rng = np.random.default_rng(12)
    nx, ny, nz = 6, 4, 2
    dx, dy = 2e-3, 3e-3
    x0, y0 = -0.005, 0.001
    kx, ky, xc, yc = oracle.mode_axes(nx, ny, x0, y0, dx, dy)
    zc = rng.standard_normal((ny, nx, nz)) + 1j * rng.standard_normal((ny, nx, nz))
    ref = np.zeros((nx, ny, nz), complex)
    for u in range(nx):
        for v in range(ny):
            xu, yv = x0 + u * dx, y0 + v * dy
            for q in range(ny):
                for p in range(nx):
                    ref[u, v] += zc[q, p] * np.exp(1j * (kx[p] * (xu - xc) + ky[q] * (yv - yc)))
    assert _rel(oracle.idft2(zc), ref) < 1e-13


# --------------------------------------------------------------------------
# whole pipeline
# --------------------------------------------------------------------------

def _grid(nx, ny, nz, dx, dz, zc, z_ref=0.0, z_focus=None):
    return ImageGrid(nx=nx, ny=ny, nz=nz, x0=-(nx // 2) * dx, y0=-(ny // 2) * dx, z0=zc - (nz // 2) * dz,
                     dx=dx, dy=dx, dz=dz, z_ref=z_ref, z_focus=zc if z_focus is None else z_focus)


def test_lateral_shift_moves_image_one_voxel():
    rng = np.random.default_rng(13)
    grid = _grid(12, 10, 4, 2e-3, 0.02, 0.3)
    tx, rx = awr1443_layout()
    pos = np.stack([rng.uniform(-0.01, 0.01, 30), rng.uniform(-0.01, 0.01, 30), rng.uniform(-3e-3, 3e-3, 30)], 1)
    freq = sweep(8)
    echo = rng.standard_normal((30, 8, 8)) + 1j * rng.standard_normal((30, 8, 8))
    o1 = oracle.reconstruct_direct(pos, tx, rx, freq, echo, grid)
    p2 = pos.copy()
    p2[:, 0] += grid.dx
    o2 = oracle.reconstruct_direct(p2, tx, rx, freq, echo, grid)
    assert _rel(o2, np.roll(o1, 1, axis=0)) < 1e-11
    p3 = pos.copy()
    p3[:, 1] -= grid.dy
    o3 = oracle.reconstruct_direct(p3, tx, rx, freq, echo, grid)
    assert _rel(o3, np.roll(o1, -1, axis=1)) < 1e-11


def test_rigid_z_translation_is_invariant():
    # moving array plane, trajectory, scene, image volume and reference depth
    # together by the same dz leaves the echo and therefore the image unchanged;
    # this fixes how the projection plane Z_0 enters the filter and the z sum.
    rng = np.random.default_rng(14)
    tx, rx = awr1443_layout()
    pos = np.stack([rng.uniform(-0.01, 0.01, 40), rng.uniform(-0.01, 0.01, 40), rng.uniform(-3e-3, 3e-3, 40)], 1)
    freq = sweep(8)
    echo = rng.standard_normal((40, 8, 8)) + 1j * rng.standard_normal((40, 8, 8))
    g1 = _grid(8, 8, 6, 2e-3, 0.02, 0.3)
    o1 = oracle.reconstruct_direct(pos, tx, rx, freq, echo, g1)
    shift = 0.0537
    g2 = _grid(8, 8, 6, 2e-3, 0.02, 0.3 + shift, z_ref=shift)
    p2 = pos.copy()
    p2[:, 2] += shift
    o2 = oracle.reconstruct_direct(p2, tx, rx, freq, echo, g2)
    assert _rel(o2, o1) < 1e-10


def test_linearity():
    rng = np.random.default_rng(15)
    grid = _grid(8, 8, 4, 2e-3, 0.02, 0.3)
    tx, rx = awr1443_layout()
    pos = np.stack([rng.uniform(-0.01, 0.01, 10), rng.uniform(-0.01, 0.01, 10), rng.uniform(-3e-3, 3e-3, 10)], 1)
    freq = sweep(6)
    e1 = rng.standard_normal((10, 8, 6)) + 1j * rng.standard_normal((10, 8, 6))
    e2 = rng.standard_normal((10, 8, 6)) + 1j * rng.standard_normal((10, 8, 6))
    f = lambda e: oracle.reconstruct_direct(pos, tx, rx, freq, e, grid)   # noqa: E731
    assert _rel(f(2.0 * e1 - 3j * e2), 2.0 * f(e1) - 3j * f(e2)) < 1e-12


def test_planes_match_full_image():
    rng = np.random.default_rng(16)
    grid = _grid(8, 6, 5, 2e-3, 0.02, 0.3)
    freq = sweep(7)
    spec = rng.standard_normal((6, 8, 7)) + 1j * rng.standard_normal((6, 8, 7))
    full = oracle.image_from_spectrum(spec, freq, grid)
    part = oracle.image_planes_from_spectrum(spec, freq, grid, [4, 1], row_chunk=4)
    assert _rel(part, full[:, :, [4, 1]]) < 1e-13


def _fwhm(profile, pitch):
    """-3 dB (half power) full width by linear interpolation around the peak."""
    a = np.abs(profile) / np.abs(profile).max()
    i = int(np.argmax(a))
    t = np.sqrt(0.5)
    l = i
    while l > 0 and a[l - 1] >= t:
        l -= 1
    r = i
    while r < len(a) - 1 and a[r + 1] >= t:
        r += 1
    xl = (l - 1) + (t - a[l - 1]) / (a[l] - a[l - 1])
    xr = r + (a[r] - t) / (a[r] - a[r + 1])
    return (xr - xl) * pitch


def test_point_spread_function_resolution():
    # Eq. (17): delta_x = lambda_c R / (2 D_x), delta_z = c / (2 B); the -3 dB
    # width of the sinc-shaped response is 0.886 delta.
    lam = oracle.C0 / 79e9
    pitch = lam / 4
    n = 64
    zt = 0.3
    grid = ImageGrid(nx=n, ny=n, nz=64, x0=-(n // 2) * pitch, y0=-(n // 2) * pitch, z0=zt - 32 * 2e-3,
                     dx=pitch, dy=pitch, dz=2e-3, z_ref=0.0, z_focus=zt)
    scan = point_scan(n, n, pitch, (0.0, 0.0, zt), 32, grid)
    img = oracle.reconstruct_direct(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.echo, grid)
    peak = np.unravel_index(np.argmax(np.abs(img)), img.shape)
    assert peak == (n // 2, n // 2, 32)
    d_aperture = n * pitch
    delta_x = lam * zt / (2 * d_aperture)
    delta_z = oracle.C0 / (2 * 4e9)
    wx = _fwhm(img[:, n // 2, 32], pitch)
    wy = _fwhm(img[n // 2, :, 32], pitch)
    wz = _fwhm(img[n // 2, n // 2, :], 2e-3)
    assert abs(wx / (0.886 * delta_x) - 1) < 0.15
    assert abs(wy / (0.886 * delta_x) - 1) < 0.15
    assert abs(wz / (0.886 * delta_z) - 1) < 0.15


def _bpa_scene(z_dev, seed=21):
    lam = oracle.C0 / 79e9
    rng = np.random.default_rng(seed)
    tx, rx = awr1443_layout()
    nxs, nys = 48, 6
    ix, iy = np.meshgrid(np.arange(nxs), np.arange(nys), indexing='ij')
    x = (ix.ravel() - (nxs - 1) / 2) * lam / 4 + rng.uniform(-lam / 16, lam / 16, ix.size)
    y = (iy.ravel() - (nys - 1) / 2) * 2 * lam + rng.uniform(-lam / 16, lam / 16, ix.size)
    z = rng.uniform(-z_dev, z_dev, ix.size)
    pos = np.stack([x, y, z], 1)
    freq = sweep(16)
    grid = ImageGrid(nx=24, ny=24, nz=8, x0=-0.024, y0=-0.024, z0=0.21, dx=2e-3, dy=2e-3, dz=0.01,
                     z_ref=0.0, z_focus=0.25)
    tgt = np.array([[-0.008, 0.006, 0.23], [0.010, -0.008, 0.27]])
    echo = synth_echo_numpy(pos, tx, rx, freq, tgt, np.array([1.0, 0.9j]))
    return pos, tx, rx, freq, echo, grid, tgt


def _local_peak(img, grid, t, r=3):
    u = int(round((t[0] - grid.x0) / grid.dx))
    v = int(round((t[1] - grid.y0) / grid.dy))
    w = int(round((t[2] - grid.z0) / grid.dz))
    sl = (slice(max(u - r, 0), u + r + 1), slice(max(v - r, 0), v + r + 1), slice(max(w - 1, 0), w + 2))
    sub = np.abs(img[sl])
    loc = np.unravel_index(np.argmax(sub), sub.shape)
    return np.array([loc[0] + sl[0].start, loc[1] + sl[1].start, loc[2] + sl[2].start]), sub.max()


def test_matches_backprojection_peaks():
    pos, tx, rx, freq, echo, grid, tgt = _bpa_scene(3e-3)
    o_b = oracle.bpa(pos, tx, rx, freq, echo, grid)
    o_r = oracle.reconstruct_direct(pos, tx, rx, freq, echo, grid)
    gb = np.array(np.unravel_index(np.argmax(np.abs(o_b)), o_b.shape))
    gr = np.array(np.unravel_index(np.argmax(np.abs(o_r)), o_r.shape))
    assert np.abs(gb - gr).max() <= 1
    for t in tgt:
        pb, _ = _local_peak(o_b, grid, t)
        pr, _ = _local_peak(o_r, grid, t)
        assert np.abs(pb - pr).max() <= 1


def test_uncompensated_reconstruction_degrades():
    # Sec. III: the RMA applied to raw multi-planar data loses focus
    pos, tx, rx, freq, echo, grid, tgt = _bpa_scene(2e-2, seed=22)
    o_c = oracle.reconstruct_direct(pos, tx, rx, freq, echo, grid, compensation=True)
    o_u = oracle.reconstruct_direct(pos, tx, rx, freq, echo, grid, compensation=False)
    for t in tgt:
        _, mc = _local_peak(o_c, grid, t)
        _, mu = _local_peak(o_u, grid, t)
        assert mu < 0.5 * mc


def test_filter_flattens_spherical_wave_spectrum():
    # Eq. (13) expands exp(-j 2k R_0)/R_0 into plane waves weighted 1/k_z
    # (Weyl's identity); the k_z factor of Eq. (15) must cancel that weight, so
    # the filtered spectrum of a point's spherical wave is flat in magnitude
    # while the raw spectrum falls as 1/k_z.  Wide-angle geometry so that k_z
    # varies by 1/cos(40 deg).
    lam = oracle.C0 / 79e9
    pitch, n, zt = lam / 4, 128, 0.025
    k = oracle.wavenumber(np.array([79e9]))
    a = (np.arange(n) - n // 2) * pitch
    yy, xx = np.meshgrid(a, a, indexing='ij')
    r0 = np.sqrt(xx ** 2 + yy ** 2 + zt ** 2)
    s = (np.exp(-2j * k[0] * r0) / r0).reshape(-1, 1)
    kx, ky, xc, yc = oracle.mode_axes(n, n, a[0], a[0], pitch, pitch)
    spec = oracle.nudft2(s, xx.ravel(), yy.ravel(), kx, ky, xc, yc)
    kz, mask = oracle.axial_wavenumber(k, kx, ky)
    filt = oracle.rma_filter(spec, kz, mask, 0.0)
    kxx, kyy = np.meshgrid(kx, ky, indexing='xy')
    reg = (kxx ** 2 + kyy ** 2) <= (2 * k[0] * np.sin(np.radians(40))) ** 2
    lk = np.log(kz[..., 0][reg])
    slope_f = np.polyfit(lk, np.log(np.abs(filt[..., 0][reg])), 1)[0]
    slope_s = np.polyfit(lk, np.log(np.abs(spec[..., 0][reg])), 1)[0]
    assert abs(slope_f) < 0.3
    assert abs(slope_s + 1.0) < 0.3


# --------------------------------------------------------------------------
# depth slabs: a reference depth per slab (Sec. V-A's depth aberrations)
# --------------------------------------------------------------------------

def test_slab_grids_partition_and_reference_depths():
    g = ImageGrid(nx=8, ny=8, nz=16, x0=0.0, y0=0.0, z0=0.1, dx=1e-3, dy=1e-3, dz=0.025, z_ref=0.0, z_focus=0.3)
    sl = oracle.slab_grids(g, 4)
    planes = np.concatenate([s.z0 + s.dz * np.arange(s.nz) for s in sl])
    np.testing.assert_allclose(planes, g.z0 + g.dz * np.arange(g.nz), rtol=0, atol=1e-15)
    assert [s.nz for s in sl] == [4, 4, 4, 4]
    np.testing.assert_allclose([s.z_focus for s in sl], [0.1375, 0.2375, 0.3375, 0.4375], rtol=0, atol=1e-15)
    with pytest.raises(ValueError):
        oracle.slab_grids(g, 3)


def test_one_slab_is_the_single_depth_image_at_the_volume_centre():
    sc = depth_pair_scan(n_side=16, n_freq=16)
    g = sc.grid
    o1 = oracle.reconstruct_slabs(sc.pos, sc.tx_xy, sc.rx_xy, sc.freq, sc.echo, g, 1)
    gc = dataclasses.replace(g, z_focus=g.z0 + 0.5 * (g.nz - 1) * g.dz)
    assert np.array_equal(o1, oracle.reconstruct_direct(sc.pos, sc.tx_xy, sc.rx_xy, sc.freq, sc.echo, gc))


def test_slab_reference_depth_removes_multistatic_residual():
    # exact round trip minus the planar model 2 R_0 + beta for the on-axis
    # near target (0.15 m) of the wide-baseline array: with R_c = 0.3 m the
    # multistatic term leaves k |d|^2/4 |1/R - 1/R_c| ~ 2.2 rad on the 4 cm
    # pairs; with the reference at the target's slab centre (0.1375 m, four
    # slabs over [0.1, 0.5)) it drops below 0.5 rad
    sc = depth_pair_scan(n_side=2, n_freq=2)
    k = float(oracle.wavenumber(np.array([79e9]))[0])
    pos = np.zeros((1, 3))
    xT, yT, xR, yR, zl = geo.tx_rx_coordinates(pos, sc.tx_xy, sc.rx_xy)
    xv, yv, dx, dy, dz = geo.virtual_samples(pos, sc.tx_xy, sc.rx_xy, 0.0)
    tgt = (0.0, 0.0, 0.15)
    r_exact = geo.round_trip_exact(xT, yT, xR, yR, zl, tgt)
    r0 = np.sqrt((xv - tgt[0]) ** 2 + (yv - tgt[1]) ** 2 + tgt[2] ** 2)
    ph_single = np.abs(k * (r_exact - 2 * r0 - geo.residual_path(dx, dy, dz, 0.0, 0.3)))
    zc = oracle.slab_grids(sc.grid, 4)[0].z_focus
    ph_slab = np.abs(k * (r_exact - 2 * r0 - geo.residual_path(dx, dy, dz, 0.0, zc)))
    assert ph_single.max() > 2.0
    assert ph_slab.max() < 0.5


def test_slab_reference_depths_refocus_a_depth_extended_scene():
    # the same residuals seen in the image: the coherent sum over the four
    # pairs of the near target falls to about cos((2.2 - 0.55) / 2) ~ 0.68 of
    # its focused value under one reference depth, and stays above 0.95 of it
    # with four slabs; both on-axis targets focus higher with slabs, and the
    # near one (lateral resolution ~10 voxels) stays on its voxel (the far
    # one's lateral response is ~30 voxels wide, too flat to locate)
    sc = depth_pair_scan()
    g = sc.grid
    o_one = oracle.reconstruct_direct(sc.pos, sc.tx_xy, sc.rx_xy, sc.freq, sc.echo, g)
    o_sl = oracle.reconstruct_slabs(sc.pos, sc.tx_xy, sc.rx_xy, sc.freq, sc.echo, g, 4)
    ratio = []
    for t in sc.targets:
        w = int(round((t[2] - g.z0) / g.dz))
        ratio.append(np.abs(o_one[16, 16, w]) / np.abs(o_sl[16, 16, w]))
    w = int(round((sc.targets[0][2] - g.z0) / g.dz))
    assert np.unravel_index(np.argmax(np.abs(o_sl[14:19, 14:19, w - 2:w + 3])), (5, 5, 5)) == (2, 2, 2)
    assert ratio[0] < 0.8
    assert ratio[1] < 1.0
