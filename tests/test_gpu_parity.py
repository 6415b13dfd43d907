"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Tolerances.  The library approximates two exact sums with NUFFTs whose kernel
width follows the plan's `tol` (default 1e-3: 4-tap Kaiser-Bessel at 2x
oversampling laterally, estimated error exp(-pi*4*sqrt(1/2)) = 1.4e-4; 6-tap
exponential-of-semicircle on the Stolt axis, 1.6e-6), with float32 data,
float32 FFTs (relative rounding ~ 6e-8 * log2(N) per pass) and float64 phase
arguments.  The image bar is the method's target, relative L2 <= 1e-3 with an
exact peak voxel; the spectrum alone must meet the same 1e-3.
"""

import numpy as np
import pytest

import oracle
from sarsynth import ImageGrid, awr1443_layout, config1_scan, sweep
from tests.sar_testutil import make_plan, peak_index, peak_ok, rel_l2, to_device

pytestmark = pytest.mark.gpu

IMAGE_TOL = 1e-3


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def tiny():
    scan = config1_scan(0)
    spec = oracle.spectrum_direct(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.echo, scan.grid)
    img = oracle.image_from_spectrum(spec, scan.freq, scan.grid)
    return scan, spec, img


def test_tiny_spectrum_matches_oracle(torch_cuda, tiny):
    scan, spec_ref, _ = tiny
    plan = make_plan(scan)
    pos, echo, sc = to_device(scan)
    spec = plan.spectrum(pos, echo).cpu().numpy()
    err = rel_l2(spec, spec_ref)
    print(f"tiny spectrum rel-L2 {err:.3e} (width {plan.info['width']})")
    assert err <= IMAGE_TOL


def test_tiny_image_matches_oracle(torch_cuda, tiny):
    scan, _, img_ref = tiny
    plan = make_plan(scan)
    pos, echo, sc = to_device(scan)
    img = plan.reconstruct(pos, echo).cpu().numpy()
    err = rel_l2(img, img_ref)
    print(f"tiny image rel-L2 {err:.3e}; peak gpu {peak_index(img)} ref {peak_index(img_ref)}")
    assert err <= IMAGE_TOL
    assert peak_ok(img, img_ref)


def test_image_from_spectrum_matches_oracle(torch_cuda):
    rng = np.random.default_rng(3)
    grid = ImageGrid(nx=64, ny=32, nz=32, x0=-0.03, y0=-0.015, z0=0.2, dx=0.03 / 32, dy=0.03 / 32,
                     dz=0.004, z_ref=0.0, z_focus=0.26)
    tx, rx = awr1443_layout()
    freq = sweep(48)
    spec = (rng.standard_normal((32, 64, 48)) + 1j * rng.standard_normal((32, 64, 48))).astype(np.complex64)
    ref = oracle.image_from_spectrum(spec.astype(np.complex128), freq, grid)
    from paper_2305_02064_amd import sar
    plan = sar.Plan(tx, rx, freq, grid, 0)
    d = torch_cuda.from_numpy(spec).cuda()
    img = plan.image_from_spectrum(d).cpu().numpy()
    err = rel_l2(img, ref)
    print(f"image_from_spectrum rel-L2 {err:.3e}")
    assert err <= IMAGE_TOL


def _ragged_scan(seed, n_pos, nf, grid, spread=1.6):
    rng = np.random.default_rng(seed)
    tx, rx = awr1443_layout()
    ext_x = grid.nx * grid.dx * spread
    ext_y = grid.ny * grid.dy * spread
    pos = np.stack([rng.uniform(-ext_x / 2, ext_x / 2, n_pos), rng.uniform(-ext_y / 2, ext_y / 2, n_pos),
                    rng.uniform(-0.01, 0.01, n_pos)], 1)
    echo = (rng.standard_normal((n_pos, 8, nf)) + 1j * rng.standard_normal((n_pos, 8, nf))).astype(np.complex64)
    from sarsynth import Scan
    return Scan(pos=pos, tx_xy=tx, rx_xy=rx, freq=sweep(nf), grid=grid, echo=echo)


@pytest.mark.parametrize("width", [3, 4, 5, 6, 7, 8])
def test_ragged_spectrum_all_widths(torch_cuda, width):
    # ragged sizes: n_pos not a multiple of anything, N_f not a multiple of 64,
    # nx != ny, samples spread beyond the image extent (periodic wrap)
    grid = ImageGrid(nx=16, ny=64, nz=8, x0=-0.008, y0=-0.03, z0=0.25, dx=1e-3, dy=0.95e-3, dz=0.01,
                     z_ref=0.0, z_focus=0.3)
    scan = _ragged_scan(40 + width, 333, 40, grid)
    ref = oracle.spectrum_direct(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.echo, grid)
    plan = make_plan(scan, kernel_width=width)
    pos, echo, _ = to_device(scan)
    spec = plan.spectrum(pos, echo).cpu().numpy()
    err = rel_l2(spec, ref)
    est = np.exp(-np.pi * width * np.sqrt(0.5))
    print(f"ragged spectrum width {width}: rel-L2 {err:.3e} (estimate {est:.1e})")
    assert err <= max(10 * est, 2e-5)


def test_ragged_image(torch_cuda):
    grid = ImageGrid(nx=16, ny=64, nz=8, x0=-0.008, y0=-0.03, z0=0.25, dx=1e-3, dy=0.95e-3, dz=0.01,
                     z_ref=0.0, z_focus=0.3)
    scan = _ragged_scan(50, 333, 40, grid)
    ref = oracle.reconstruct_direct(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.echo, grid)
    plan = make_plan(scan)
    pos, echo, _ = to_device(scan)
    img = plan.reconstruct(pos, echo).cpu().numpy()
    err = rel_l2(img, ref)
    print(f"ragged image rel-L2 {err:.3e}")
    assert err <= IMAGE_TOL


@pytest.mark.parametrize("nx,ny", [(1024, 8), (2048, 8), (8, 1024), (8, 2048)])
def test_largest_transform_lengths(torch_cuda, nx, ny):
    # lateral grids of 2048 and 4096 cells (the longest FFT passes, each its own
    # instantiation) along x and along y, image against the oracle
    grid = ImageGrid(nx=nx, ny=ny, nz=2, x0=-nx / 2 * 1e-3, y0=-ny / 2 * 1e-3, z0=0.25, dx=1e-3, dy=1e-3,
                     dz=0.01, z_ref=0.0, z_focus=0.3)
    scan = _ragged_scan(70 + nx + ny, 97, 6, grid)
    ref = oracle.reconstruct_direct(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.echo, grid)
    plan = make_plan(scan)
    assert max(plan.info["mx"], plan.info["my"]) == 2 * max(nx, ny)
    pos, echo, _ = to_device(scan)
    img = plan.reconstruct(pos, echo).cpu().numpy()
    plan.close()
    err = rel_l2(img, ref)
    print(f"transform lengths {plan.info['mx']} x {plan.info['my']}: image rel-L2 {err:.3e}")
    assert err <= IMAGE_TOL


def test_scan_of_more_than_1024_count_chunks(torch_cuda):
    # a 2048 x 2048 image on a 4096 x 4096 grid: 16.8 M per-cell counts, more
    # than 1024 chunks of 4096, so the cell-start scan takes its three-kernel
    # form (smaller grids take the two-kernel one); spectrum at sampled
    # entries against exact sums over every virtual sample
    grid = ImageGrid(nx=2048, ny=2048, nz=2, x0=-1.024, y0=-1.024, z0=0.25, dx=1e-3, dy=1e-3, dz=0.01,
                     z_ref=0.0, z_focus=0.3)
    scan = _ragged_scan(2222, 301, 2, grid)
    plan = make_plan(scan)
    assert plan.info["mx"] * plan.info["my"] > 1024 * 4096
    pos, echo, _ = to_device(scan)
    spec = plan.spectrum(pos, echo).cpu().numpy()
    plan.close()
    rng = np.random.default_rng(5)
    ne = 128
    qi = rng.integers(0, grid.ny, ne)
    pi = rng.integers(0, grid.nx, ne)
    fi = rng.integers(0, 2, ne)
    k = oracle.wavenumber(scan.freq)
    xv, yv, dxx, dyy, dzz = oracle.virtual_samples(scan.pos, scan.tx_xy, scan.rx_xy, grid.z_ref)
    beta = oracle.residual_path(dxx, dyy, dzz, grid.z_ref, grid.z_focus).ravel()
    kx, ky, xc, yc = oracle.mode_axes(grid.nx, grid.ny, grid.x0, grid.y0, grid.dx, grid.dy)
    shat = oracle.compensate(scan.echo.reshape(-1, 2), k, beta)
    ref = oracle.nudft2_entries(shat, xv.ravel(), yv.ravel(), kx[pi], ky[qi], fi, xc, yc)
    err = rel_l2(spec[qi, pi, fi], ref)
    print(f"4096 x 4096 grid, {ne} sampled entries: rel-L2 {err:.3e}")
    assert err <= IMAGE_TOL


@pytest.mark.parametrize("nx,ny", [(72, 100), (75, 81), (150, 250), (250, 64), (135, 243), (125, 225)])
def test_mixed_radix_image_sides(torch_cuda, nx, ny):
    # image sides of the form 2^a 3^b 5^c, odd ones included: oversampled grids
    # of 2^a 3^b 5^c cells (multiples of 8), the mixed-radix line transforms,
    # the odd-length centred crop and the shifted, phase-corrected inverse
    grid = ImageGrid(nx=nx, ny=ny, nz=8, x0=-(nx // 2) * 1e-3, y0=-(ny // 2) * 1e-3, z0=0.25, dx=1e-3, dy=1e-3,
                     dz=0.01, z_ref=0.0, z_focus=0.3)
    scan = _ragged_scan(500 + nx + ny, 149, 12, grid)
    ref = oracle.reconstruct_direct(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.echo, grid)
    pos, echo, _ = to_device(scan)
    # oversampling 2 (mixed-radix grids for most sides), then the automatic
    # choice (a power-of-two grid between 1.5 n and 2 n where there is one)
    for up in (2.0, 0.0):
        plan = make_plan(scan, upsample=up)
        img = plan.reconstruct(pos, echo).cpu().numpy()
        info = plan.info
        plan.close()
        err = rel_l2(img, ref)
        print(f"sides {nx} x {ny}, upsample {up} (grid {info['mx']} x {info['my']}, width {info['width']}): "
              f"image rel-L2 {err:.3e}")
        assert info["mx"] % 8 == 0 and info["my"] % 8 == 0
        if up == 2.0:
            assert info["mx"] >= 2 * nx and info["my"] >= 2 * ny
        else:
            assert info["mx"] >= 1.5 * nx and info["my"] >= 1.5 * ny
        assert err <= IMAGE_TOL
        assert peak_ok(img, ref)


@pytest.mark.parametrize("n,grid", [(32, 64), (96, 192), (150, 256), (162, 256), (100, 200), (512, 1024), (75, 128)])
def test_automatic_oversampling_prefers_a_power_of_two(torch_cuda, n, grid):
    # upsample 0: a power of two in [1.5 n, 2 n] if there is one, else the
    # 5-smooth grid of oversampling 2; the kernel width follows the smaller
    # oversampling (5 taps at 256 / 150, 4 at 2)
    from paper_2305_02064_amd import sar
    g = ImageGrid(nx=n, ny=n, nz=8, x0=-0.05, y0=-0.05, z0=0.25, dx=1e-3, dy=1e-3, dz=0.01, z_ref=0.0, z_focus=0.3)
    plan = sar.Plan(*awr1443_layout(), sweep(16), g, 10)
    info = plan.info
    plan.close()
    assert info["mx"] == grid and info["my"] == grid
    sigma = grid / n
    assert info["width"] == (4 if sigma >= 2 else 5)


@pytest.mark.parametrize("upsample", [1.25, 1.5])
def test_oversampling_below_two(torch_cuda, tiny, upsample):
    # sigma in [1.25, 2): grids of 2^a 3^b 5^c cells (40 and 48 cells
    # for 32 voxels), kernel widths from the plan's tolerance
    scan, spec_ref, img_ref = tiny
    plan = make_plan(scan, upsample=upsample)
    pos, echo, _ = to_device(scan)
    spec = plan.spectrum(pos, echo).cpu().numpy()
    img = plan.reconstruct(pos, echo).cpu().numpy()
    info = plan.info
    e_s, e_i = rel_l2(spec, spec_ref), rel_l2(img, img_ref)
    print(f"upsample {upsample}: grid {info['mx']} x {info['my']}, sigma {info['sigma_x']:.3f}, width "
          f"{info['width']}: spectrum {e_s:.3e}, image {e_i:.3e}")
    assert info["sigma_x"] >= upsample and info["sigma_x"] < 2
    assert e_s <= IMAGE_TOL and e_i <= IMAGE_TOL
    assert peak_ok(img, img_ref)


def test_long_sweep(torch_cuda):
    # 700 frequencies: each Stolt lane's run spans several load batches with a
    # partial last one, and the gridding's frequency chunks end mid-wave
    grid = ImageGrid(nx=16, ny=16, nz=8, x0=-0.008, y0=-0.008, z0=0.25, dx=1e-3, dy=1e-3, dz=0.01,
                     z_ref=0.0, z_focus=0.3)
    scan = _ragged_scan(91, 61, 700, grid)
    ref = oracle.reconstruct_direct(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.echo, grid)
    plan = make_plan(scan)
    pos, echo, _ = to_device(scan)
    img = plan.reconstruct(pos, echo).cpu().numpy()
    plan.close()
    err = rel_l2(img, ref)
    print(f"700-frequency sweep: image rel-L2 {err:.3e}")
    assert err <= IMAGE_TOL


@pytest.mark.parametrize("n_pos", [1, 37])
def test_other_array_layout(torch_cuda, n_pos):
    # 3 Tx x 5 Rx at irregular offsets (15 pairs, pair = t * 5 + r), one shot or
    # a few: the pair tables and the virtual-sample indexing beyond 2 x 4
    from sarsynth import Scan
    rng = np.random.default_rng(300 + n_pos)
    tx = rng.uniform(-0.01, 0.01, (3, 2))
    rx = rng.uniform(-0.01, 0.01, (5, 2))
    grid = ImageGrid(nx=16, ny=16, nz=8, x0=-0.008, y0=-0.008, z0=0.25, dx=1e-3, dy=1e-3, dz=0.01,
                     z_ref=0.0, z_focus=0.3)
    pos = np.stack([rng.uniform(-0.01, 0.01, n_pos), rng.uniform(-0.01, 0.01, n_pos),
                    rng.uniform(-0.005, 0.005, n_pos)], 1)
    nf = 24
    echo = (rng.standard_normal((n_pos, 15, nf)) + 1j * rng.standard_normal((n_pos, 15, nf))).astype(np.complex64)
    scan = Scan(pos=pos, tx_xy=tx, rx_xy=rx, freq=sweep(nf), grid=grid, echo=echo)
    ref = oracle.reconstruct_direct(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.echo, grid)
    plan = make_plan(scan)
    pos_d, echo_d, _ = to_device(scan)
    img = plan.reconstruct(pos_d, echo_d).cpu().numpy()
    plan.close()
    err = rel_l2(img, ref)
    print(f"3 x 5 array, {n_pos} shots: image rel-L2 {err:.3e}")
    assert err <= IMAGE_TOL


def test_single_frequency(torch_cuda):
    # a one-frequency sweep (a single-frequency hologram): one valid lane per
    # gridding frequency chunk, one sample per Stolt column
    grid = ImageGrid(nx=16, ny=16, nz=4, x0=-0.008, y0=-0.008, z0=0.25, dx=1e-3, dy=1e-3, dz=0.01,
                     z_ref=0.0, z_focus=0.3)
    scan = _ragged_scan(97, 45, 1, grid)
    ref = oracle.reconstruct_direct(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.echo, grid)
    plan = make_plan(scan)
    pos, echo, _ = to_device(scan)
    img = plan.reconstruct(pos, echo).cpu().numpy()
    plan.close()
    err = rel_l2(img, ref)
    print(f"single-frequency sweep: image rel-L2 {err:.3e}")
    assert err <= IMAGE_TOL


def test_no_compensation_flag(torch_cuda, tiny):
    from paper_2305_02064_amd import sar
    scan, _, _ = tiny
    ref = oracle.reconstruct_direct(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.echo, scan.grid,
                                    compensation=False)
    plan = make_plan(scan, flags=sar.SAR_NO_COMPENSATION)
    pos, echo, _ = to_device(scan)
    img = plan.reconstruct(pos, echo).cpu().numpy()
    err = rel_l2(img, ref)
    print(f"uncompensated image rel-L2 {err:.3e}")
    assert err <= IMAGE_TOL


@pytest.mark.parametrize("nz", [16, 1])
def test_stolt_jacobian_flag(torch_cuda, tiny, nz):
    # SAR_STOLT_DCF: filter factor k_z times dk_z/dk = 4k/k_z, in the oracle
    # (rma_filter(dcf=True)) and in the Stolt kernel (3-D) and the plane sum (nz = 1)
    from paper_2305_02064_amd import sar
    scan, _, _ = tiny
    g = scan.grid if nz > 1 else _plane_grid(scan.grid, 0.3)
    ref = oracle.reconstruct_direct(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.echo, g, dcf=True)
    plan = sar.Plan(scan.tx_xy, scan.rx_xy, scan.freq, g, scan.n_pos, flags=sar.SAR_STOLT_DCF)
    pos, echo, _ = to_device(scan)
    img = plan.reconstruct(pos, echo).cpu().numpy()
    err = rel_l2(img, ref)
    print(f"Stolt Jacobian image (nz {nz}) rel-L2 {err:.3e}")
    assert err <= IMAGE_TOL
    assert peak_ok(img, ref)
    plain = oracle.reconstruct_direct(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.echo, g)
    assert rel_l2(plain, ref) > 0.05   # the flag changes the image


def test_amplitude_flag(torch_cuda, tiny):
    # SAR_AMPLITUDE: each sample also scaled by R^T R^R / R_0^2 at z_focus
    # (oracle.amplitude_factor), folded into the gridding weights
    from paper_2305_02064_amd import sar
    scan, _, _ = tiny
    ref = oracle.reconstruct_direct(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.echo, scan.grid,
                                    amplitude=True)
    plan = sar.Plan(scan.tx_xy, scan.rx_xy, scan.freq, scan.grid, scan.n_pos, flags=sar.SAR_AMPLITUDE)
    pos, echo, _ = to_device(scan)
    img = plan.reconstruct(pos, echo).cpu().numpy()
    plan.close()
    err = rel_l2(img, ref)
    print(f"amplitude half image rel-L2 {err:.3e}")
    assert err <= IMAGE_TOL
    assert peak_ok(img, ref)
    plain = oracle.reconstruct_direct(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.echo, scan.grid)
    assert rel_l2(plain, ref) > 3e-3   # the flag changes the image


def test_clustered_scan_matches_oracle(torch_cuda):
    # 4608 of 5120 shots at one position: eight cells of 4608 samples each
    # (more than one 4096-sample tile of the radix sort), the tiles over them
    # walk long runs; the image must still match the oracle and be reproducible.
    # With nine tenths of the samples on eight virtual elements the lateral
    # NUFFT error is that of a few single points, not the average over spread
    # samples that the tolerance is calibrated on (a single point at a poor
    # sub-cell offset reaches about 8e-4 per axis with the 4-tap kernel), so
    # this plan asks for tol 1e-4 (5 taps) to meet the 1e-3 image bar.
    from sarsynth import clustered_scan
    scan = clustered_scan(0)
    ref = oracle.reconstruct_direct(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.echo, scan.grid)
    plan = make_plan(scan, tol=1e-4)
    pos, echo, _ = to_device(scan)
    a = plan.reconstruct(pos, echo).cpu().numpy()
    b = plan.reconstruct(pos, echo).cpu().numpy()
    err = rel_l2(a, ref)
    print(f"clustered scan ({scan.n_pos} shots, 4608 at one position): rel-L2 {err:.3e}")
    assert err <= IMAGE_TOL
    assert peak_ok(a, ref)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("width,nf", [(4, 32), (4, 160), (5, 160)])
def test_clustered_scan_split_unions(torch_cuda, width, nf):
    # the four-wave gridding kernel splits the unions over the dwell cells
    # (over 4608 samples each, parts of 2048) into overflow workgroups and adds
    # their partial grids in part order: equal to the unsplit one-wave tile up
    # to summation order, reproducible, and at the oracle's image (the 4-tap
    # kernel's single-point error, see the test above, bounds the distance)
    from sarsynth import clustered_scan
    scan = clustered_scan(0, n_freq=nf)
    ref = oracle.reconstruct_direct(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.echo, scan.grid)
    plan = make_plan(scan, kernel_width=width)
    assert plan.info["width"] == width
    pos, echo, _ = to_device(scan)
    plan.set_grid_tile(3)
    a = plan.reconstruct(pos, echo).cpu().numpy()
    b = plan.reconstruct(pos, echo).cpu().numpy()
    plan.set_grid_tile(0)
    c = plan.reconstruct(pos, echo).cpu().numpy()
    err, same = rel_l2(a, ref), rel_l2(a, c)
    print(f"clustered scan, width {width}, {nf} frequencies, split unions: vs unsplit tile {same:.2e}, "
          f"vs oracle {err:.3e}")
    assert np.array_equal(a, b)
    # float32 sums of ~4600 samples per dwell cell in another order: about
    # sqrt(4600) x 2^-24 ~ 4e-6 apart at most
    assert same <= 5e-6
    assert err <= 3e-3
    assert peak_ok(a, ref)


def test_empty_scan_gives_zero_image(torch_cuda, tiny):
    scan, _, _ = tiny
    plan = make_plan(scan)
    pos, echo, _ = to_device(scan)
    img = plan.new_image()
    img.fill_(1.0)
    from paper_2305_02064_amd import sar
    sar.sar_reconstruct(plan.handle, pos, 0, echo, 1.0, img, plan.ws)
    assert float(img.abs().max().item()) == 0.0


def test_deterministic(torch_cuda, tiny):
    scan, _, _ = tiny
    plan = make_plan(scan)
    pos, echo, _ = to_device(scan)
    a = plan.reconstruct(pos, echo).cpu().numpy()
    b = plan.reconstruct(pos, echo).cpu().numpy()
    assert np.array_equal(a, b)


def test_half_echo_precision(torch_cuda, tiny):
    # FP16 echo storage with one per-scan scale; phase arguments stay FP64
    from paper_2305_02064_amd import sar
    scan, _, img_ref = tiny
    plan = make_plan(scan, echo_type=sar.SAR_ECHO_F16X2)
    pos, eh, scale = to_device(scan, half=True)
    img = plan.reconstruct(pos, eh, echo_scale=scale).cpu().numpy()
    err = rel_l2(img, img_ref)
    print(f"fp16-echo image rel-L2 {err:.3e}, peak {peak_index(img)} ref {peak_index(img_ref)}")
    assert err <= IMAGE_TOL
    assert peak_ok(img, img_ref)


@pytest.mark.parametrize("nz", [2, 16, 64, 128, 256, 512])
def test_stolt_grid_sizes(torch_cuda, nz):
    # every Stolt grid size (64 .. 1024 cells) against the direct non-uniform sum
    rng = np.random.default_rng(100 + nz)
    grid = ImageGrid(nx=16, ny=8, nz=nz, x0=-0.008, y0=-0.004, z0=0.25, dx=1e-3, dy=1e-3,
                     dz=0.2 / nz, z_ref=0.0, z_focus=0.3)
    tx, rx = awr1443_layout()
    freq = sweep(24)
    spec = (rng.standard_normal((8, 16, 24)) + 1j * rng.standard_normal((8, 16, 24))).astype(np.complex64)
    ref = oracle.image_from_spectrum(spec.astype(np.complex128), freq, grid)
    from paper_2305_02064_amd import sar
    plan = sar.Plan(tx, rx, freq, grid, 0)
    img = plan.image_from_spectrum(torch_cuda.from_numpy(spec).cuda()).cpu().numpy()
    err = rel_l2(img, ref)
    print(f"Stolt nz={nz} (grid {plan.info['mz']}): rel-L2 {err:.3e}")
    assert err <= 1e-4


@pytest.mark.parametrize("width,nf", [(4, 40), (4, 200), (5, 40), (5, 200), (6, 200)])
def test_gridding_tiles_agree(torch_cuda, width, nf):
    # every tile configuration compiled for the width (4x4 cells, 2
    # frequencies per lane; 8x8 cells, 1 frequency; 8x4 cells, 2 frequencies;
    # the four-wave 8x8 union, 2 frequencies, 3-5 taps) against each other and
    # the oracle; 200 frequencies leave a ragged last frequency chunk
    grid = ImageGrid(nx=16, ny=32, nz=8, x0=-0.008, y0=-0.015, z0=0.25, dx=1e-3, dy=0.95e-3, dz=0.01,
                     z_ref=0.0, z_focus=0.3)
    scan = _ragged_scan(70 + width + nf, 211, nf, grid)
    ref = oracle.spectrum_direct(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.echo, grid)
    plan = make_plan(scan, kernel_width=width)
    pos, echo, _ = to_device(scan)
    from paper_2305_02064_amd import sar
    tiles, specs = [], []
    for tile in (0, 1, 2, 3):
        try:
            plan.set_grid_tile(tile)
        except sar.SarError as e:   # not compiled for this width
            assert e.status == sar.SAR_ERR_UNSUPPORTED
            continue
        assert plan.info["grid_tile"] == tile
        tiles.append(tile)
        specs.append(plan.spectrum(pos, echo).cpu().numpy())
    assert len(tiles) >= 2
    est = np.exp(-np.pi * width * np.sqrt(0.5))
    for tile, spec in zip(tiles, specs):
        err = rel_l2(spec, ref)
        print(f"tile {tile} width {width} nf {nf}: rel-L2 {err:.3e}")
        assert err <= max(10 * est, 2e-5)
        assert rel_l2(spec, specs[0]) <= 1e-6


@pytest.mark.parametrize("width,nf", [(3, 200), (5, 200), (5, 199)])
def test_union_tile_half_precision_echo(torch_cuda, width, nf):
    # FP16 echo storage (half pairs staged in the first half of a sample's LDS
    # slot) through the four-wave union at 3 and 5 taps, and an odd sweep
    # (single-value stores): equal to the one-wave tile up to summation order
    from paper_2305_02064_amd import sar
    grid = ImageGrid(nx=16, ny=32, nz=8, x0=-0.008, y0=-0.015, z0=0.25, dx=1e-3, dy=0.95e-3, dz=0.01,
                     z_ref=0.0, z_focus=0.3)
    scan = _ragged_scan(900 + width + nf, 211, nf, grid)
    plan = make_plan(scan, kernel_width=width, echo_type=sar.SAR_ECHO_F16X2)
    pos, echo, scale = to_device(scan, half=True)
    out = []
    for tile in (0, 3):
        plan.set_grid_tile(tile)
        out.append(plan.spectrum(pos, echo, echo_scale=scale).cpu().numpy())
    plan.close()
    ref = oracle.spectrum_direct(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.echo, grid)
    d, e = rel_l2(out[1], out[0]), rel_l2(out[1], ref)
    print(f"FP16 echo, width {width}, nf {nf}: union vs one-wave tile {d:.2e}, vs oracle {e:.3e}")
    assert d <= 1e-6
    # the NUFFT estimate, or FP16 rounding of random values (~3e-4 rms)
    assert e <= max(10 * np.exp(-np.pi * width * np.sqrt(0.5)), 1e-3)


def test_autotune_keeps_a_working_tile(torch_cuda, tiny):
    from paper_2305_02064_amd import sar
    scan, _, img_ref = tiny
    plan = make_plan(scan)
    pos, echo, _ = to_device(scan)
    tile = plan.autotune(pos, echo)
    assert tile in (0, 1, 2, 3) and plan.info["grid_tile"] == tile
    img = plan.reconstruct(pos, echo).cpu().numpy()
    assert rel_l2(img, img_ref) <= IMAGE_TOL
    plan.set_grid_tile(tile)
    assert np.array_equal(plan.reconstruct(pos, echo).cpu().numpy(), img)
    wide = make_plan(scan, kernel_width=8)
    with pytest.raises(sar.SarError) as ei:
        wide.set_grid_tile(1)
    assert ei.value.status == sar.SAR_ERR_UNSUPPORTED


def _plane_grid(g, z):
    return ImageGrid(nx=g.nx, ny=g.ny, nz=1, x0=g.x0, y0=g.y0, z0=z, dx=g.dx, dy=g.dy, dz=g.dz,
                     z_ref=g.z_ref, z_focus=g.z_focus)


def test_single_plane_image_matches_oracle(torch_cuda, tiny):
    # the 2-D image at a known depth (nz = 1): one exact sum over frequency per column
    scan, _, _ = tiny
    g2 = _plane_grid(scan.grid, 0.3)
    ref = oracle.reconstruct_direct(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.echo, g2)
    from paper_2305_02064_amd import sar
    plan = sar.Plan(scan.tx_xy, scan.rx_xy, scan.freq, g2, scan.n_pos)
    pos, echo, _ = to_device(scan)
    img = plan.reconstruct(pos, echo).cpu().numpy()
    assert img.shape == (g2.nx, g2.ny, 1)
    err = rel_l2(img, ref)
    print(f"2-D plane image rel-L2 {err:.3e}; peak gpu {peak_index(img)} ref {peak_index(ref)}")
    assert err <= IMAGE_TOL
    assert peak_ok(img, ref)


def test_single_plane_equals_plane_of_3d_image(torch_cuda, tiny):
    scan, _, _ = tiny
    g = scan.grid
    w = 8
    g2 = _plane_grid(g, g.z0 + w * g.dz)
    from paper_2305_02064_amd import sar
    p3 = make_plan(scan)
    p2 = sar.Plan(scan.tx_xy, scan.rx_xy, scan.freq, g2, scan.n_pos)
    pos, echo, _ = to_device(scan)
    a = p3.reconstruct(pos, echo)[:, :, w].cpu().numpy()
    b = p2.reconstruct(pos, echo)[:, :, 0].cpu().numpy()
    err = rel_l2(b, a)
    print(f"2-D plane vs plane {w} of the 3-D image: rel-L2 {err:.3e}")
    assert err <= 1e-4
