"""Parity at the full size of the large freehand scan (512 x 256 shots x 8 pairs
x 256 frequencies -> 512 x 256 x 256 voxels), in the launch configuration the
benchmark times.  The oracle cannot afford whole images at this size, so:

* dense echo: the spectrum (steps a0-a3) at 256 sampled (k_x, k_y, f) entries,
  each an exact sum over all 1 048 576 virtual samples;
* sparse echo (every shot's echo zero except 24 shots): whole z planes of the
  image -- the zero shots still go through geometry, sorting and gridding on
  the GPU, while the oracle sums only the non-zero ones;
* linearity of the full path on dense echoes (holds at any size);
* whole (k_x, k_y) planes of the dense spectrum at three frequencies, and the
  back end (steps a4-a6) on a whole image from a dense oracle spectrum.
"""

import numpy as np
import pytest

import oracle
from tests.sar_testutil import make_plan, peak_index, peak_ok, rel_l2, to_device

pytestmark = pytest.mark.gpu

IMAGE_TOL = 1e-3


@pytest.fixture(scope="module")
def big():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from sarsynth import config2_scan
    scan = config2_scan(0, device=torch.device("cuda", 0))
    plan = make_plan(scan)
    pos, echo, _ = to_device(scan)
    return scan, plan, pos, echo


def test_fullsize_spectrum_sampled_entries(big):
    scan, plan, pos, echo = big
    g = scan.grid
    spec = plan.spectrum(pos, echo)
    rng = np.random.default_rng(1)
    ne = 256
    qi = rng.integers(0, g.ny, ne)
    pi = rng.integers(0, g.nx, ne)
    fi = rng.integers(0, scan.n_freq, ne)
    got = spec.cpu().numpy()[qi, pi, fi]
    # oracle: exact sums over every virtual sample for the sampled entries
    k = oracle.wavenumber(scan.freq)
    xv, yv, dxx, dyy, dzz = oracle.virtual_samples(scan.pos, scan.tx_xy, scan.rx_xy, g.z_ref)
    beta = oracle.residual_path(dxx, dyy, dzz, g.z_ref, g.z_focus).ravel()
    kx, ky, xc, yc = oracle.mode_axes(g.nx, g.ny, g.x0, g.y0, g.dx, g.dy)
    uf = np.unique(fi)
    e_host = echo[:, :, uf].cpu().numpy().reshape(-1, len(uf))
    shat = oracle.compensate(e_host, k[uf], beta)
    col = np.searchsorted(uf, fi)
    ref = oracle.nudft2_entries(shat, xv.ravel(), yv.ravel(), kx[pi], ky[qi], col, xc, yc)
    err = rel_l2(got, ref)
    print(f"full-size spectrum, {ne} sampled entries: rel-L2 {err:.3e}")
    assert err <= IMAGE_TOL


def test_fullsize_sparse_echo_image_planes(big):
    import torch
    scan, plan, pos, echo = big
    g = scan.grid
    rng = np.random.default_rng(2)
    shots = np.sort(rng.choice(scan.n_pos, 24, replace=False))
    e_sparse = torch.zeros_like(echo)
    e_sparse[torch.from_numpy(shots).cuda()] = echo[torch.from_numpy(shots).cuda()]
    img = plan.reconstruct(pos, e_sparse)
    w_list = [3, 100, 128, 250]
    got = img[:, :, w_list].cpu().numpy()
    e_host = e_sparse[torch.from_numpy(shots).cuda()].cpu().numpy()
    spec = oracle.spectrum_direct(scan.pos[shots], scan.tx_xy, scan.rx_xy, scan.freq, e_host, g)
    ref = oracle.image_planes_from_spectrum(spec, scan.freq, g, w_list)
    err = rel_l2(got, ref)
    print(f"full-size sparse-echo image planes {w_list}: rel-L2 {err:.3e}")
    assert err <= IMAGE_TOL
    for j in range(len(w_list)):
        assert rel_l2(got[:, :, j], ref[:, :, j]) <= 2 * IMAGE_TOL


def test_fullsize_linearity(big):
    scan, plan, pos, echo = big
    import torch
    g = torch.Generator(device=echo.device)
    g.manual_seed(5)
    e2 = torch.complex(torch.randn(echo.shape, generator=g, device=echo.device),
                       torch.randn(echo.shape, generator=g, device=echo.device)) * echo.abs().mean()
    a = plan.reconstruct(pos, echo).clone()
    b = plan.reconstruct(pos, e2).clone()
    c = plan.reconstruct(pos, (echo * 0.5 - 2j * e2).contiguous())
    err = float(((c - (0.5 * a - 2j * b)).abs().norm() / c.abs().norm()).item())
    print(f"full-size linearity residual {err:.3e}")
    assert err <= 1e-5


def test_fullsize_spectrum_whole_planes(big):
    # whole (k_x, k_y) planes of the dense large-scan spectrum at the first,
    # middle and last frequency, each an exact sum over all 1 048 576 virtual
    # samples (direct 2-D NUDFT, about 15 s of host time per plane)
    scan, plan, pos, echo = big
    g = scan.grid
    spec = plan.spectrum(pos, echo)
    k = oracle.wavenumber(scan.freq)
    xv, yv, dxx, dyy, dzz = oracle.virtual_samples(scan.pos, scan.tx_xy, scan.rx_xy, g.z_ref)
    beta = oracle.residual_path(dxx, dyy, dzz, g.z_ref, g.z_focus).ravel()
    kx, ky, xc, yc = oracle.mode_axes(g.nx, g.ny, g.x0, g.y0, g.dx, g.dy)
    for f in (0, scan.n_freq // 2, scan.n_freq - 1):
        got = spec[:, :, f].cpu().numpy()
        e_host = echo[:, :, f].cpu().numpy().reshape(-1, 1)
        shat = oracle.compensate(e_host, k[f:f + 1], beta)
        ref = oracle.nudft2(shat, xv.ravel(), yv.ravel(), kx, ky, xc, yc, block=32768)[:, :, 0]
        err = rel_l2(got, ref)
        print(f"full-size spectrum plane f{f}: rel-L2 {err:.3e}", flush=True)
        assert err <= IMAGE_TOL


def test_fullsize_back_end_whole_image(big):
    # steps a4-a6 at full size on a whole 512 x 256 x 256 image: the input
    # spectrum is the oracle's own (dense, structured: 24 shots of the scan),
    # the reference image the oracle's, computed plane group by plane group on
    # the host's cores
    import concurrent.futures as cf
    import os
    import torch
    scan, plan, pos, echo = big
    g = scan.grid
    rng = np.random.default_rng(3)
    shots = np.sort(rng.choice(scan.n_pos, 24, replace=False))
    e_host = echo[torch.from_numpy(shots).cuda()].cpu().numpy()
    spec = oracle.spectrum_direct(scan.pos[shots], scan.tx_xy, scan.rx_xy, scan.freq, e_host, g)
    got = plan.image_from_spectrum(torch.from_numpy(spec.astype(np.complex64)).cuda()).cpu().numpy()
    groups = np.array_split(np.arange(g.nz), max(1, min(32, len(os.sched_getaffinity(0)))))
    ref = np.zeros((g.nx, g.ny, g.nz), np.complex128)
    with cf.ThreadPoolExecutor(max_workers=len(groups)) as ex:
        parts = list(ex.map(lambda w: (w, oracle.image_planes_from_spectrum(spec, scan.freq, g, list(w))), groups))
    for w, im in parts:
        ref[:, :, w] = im
    err = rel_l2(got, ref)
    pg, pr = peak_index(got), peak_index(ref)
    print(f"full-size back end, whole image: rel-L2 {err:.3e}, peak {pg} vs {pr}", flush=True)
    assert err <= IMAGE_TOL
    assert peak_ok(got, ref)
