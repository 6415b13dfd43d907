"""GPU tests of depth-slab plans (n_slabs > 1: a reference depth per slab of
planes, through the C ABI).

Checked against the FP64 oracle's reconstruct_slabs (each slab is the direct
reconstruction of its planes compensated with the slab's own reference depth):
relative L2 <= 1e-3 with the exact peak voxel, on the wide-baseline two-depth
scene and on the tiny freehand scan.  Also: the slabs refocus the near target
of the two-depth scene as in the oracle; a slab plan inside a fused batch,
and served beside a single-depth plan, equals the plain call; a depth-slab
plan refuses the single-spectrum calls.  The amplitude half of the
compensation (SAR_AMPLITUDE: each sample scaled by R^T R^R / R_0^2 at its slab's
reference depth) matches the oracle's on the two-depth scene with tilted shots,
with one reference depth and with four slabs.
"""

import numpy as np
import pytest

import oracle
from sarsynth import config1_scan, depth_pair_scan, synth_echo_numpy
from tests.sar_testutil import peak_ok, rel_l2, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _plan(sc, **kw):
    from paper_2305_02064_amd import sar
    return sar.Plan(sc.tx_xy, sc.rx_xy, sc.freq, sc.grid, sc.n_pos, **kw)


@pytest.mark.parametrize("n_slabs", [2, 4, 16])
def test_depth_pair_slabs_match_oracle(torch_cuda, n_slabs):
    sc = depth_pair_scan()
    pos, echo, _ = to_device(sc)
    plan = _plan(sc, n_slabs=n_slabs)
    try:
        assert plan.info["n_slabs"] == n_slabs
        img = plan.reconstruct(pos, echo).cpu().numpy()
    finally:
        plan.close()
    ref = oracle.reconstruct_slabs(sc.pos, sc.tx_xy, sc.rx_xy, sc.freq, sc.echo, sc.grid, n_slabs)
    err = rel_l2(img, ref)
    print(f"depth-pair scene, {n_slabs} slabs: rel-L2 {err:.3e}")
    assert err <= 1e-3
    assert peak_ok(img, ref)


def test_slabs_refocus_near_target(torch_cuda):
    sc = depth_pair_scan()
    pos, echo, _ = to_device(sc)
    one, four = _plan(sc), _plan(sc, n_slabs=4)
    try:
        a = np.abs(one.reconstruct(pos, echo).cpu().numpy())
        b = np.abs(four.reconstruct(pos, echo).cpu().numpy())
    finally:
        one.close()
        four.close()
    g = sc.grid
    ratios = []
    for t in sc.targets:
        w = int(round((t[2] - g.z0) / g.dz))
        ratios.append(float(a[16, 16, w] / b[16, 16, w]))
    print(f"single-depth / 4-slab magnitude at the targets: {ratios[0]:.3f} (0.15 m), {ratios[1]:.3f} (0.45 m)")
    assert ratios[0] < 0.8
    assert ratios[1] < 1.0


def test_tiny_scan_slabs_match_oracle(torch_cuda):
    sc = config1_scan(0)
    pos, echo, _ = to_device(sc)
    plan = _plan(sc, n_slabs=2)
    try:
        img = plan.reconstruct(pos, echo).cpu().numpy()
    finally:
        plan.close()
    ref = oracle.reconstruct_slabs(sc.pos, sc.tx_xy, sc.rx_xy, sc.freq, sc.echo, sc.grid, 2)
    err = rel_l2(img, ref)
    print(f"tiny scan, 2 slabs: rel-L2 {err:.3e}")
    assert err <= 1e-3
    assert peak_ok(img, ref)


def test_slab_plan_in_batch_equals_plain(torch_cuda):
    from paper_2305_02064_amd import sar
    scans = [depth_pair_scan(), config1_scan(0)]
    plans = [_plan(scans[0], n_slabs=4), _plan(scans[1])]
    dev = [to_device(sc) for sc in scans]
    try:
        refs = [p.reconstruct(d[0], d[1]).clone() for p, d in zip(plans, dev)]
        b = sar.Batch(plans)
        try:
            for _ in range(2):
                imgs = b.reconstruct([d[0] for d in dev], [d[1] for d in dev])
                torch_cuda.cuda.synchronize()
                for k, (img, ref) in enumerate(zip(imgs, refs)):
                    assert rel_l2(img.cpu().numpy(), ref.cpu().numpy()) <= 1e-6, k
        finally:
            b.close()
    finally:
        for p in plans:
            p.close()


def test_slab_plan_refuses_single_spectrum_calls(torch_cuda):
    from paper_2305_02064_amd import sar
    sc = depth_pair_scan()
    pos, echo, _ = to_device(sc)
    plan = _plan(sc, n_slabs=2)
    try:
        with pytest.raises(sar.SarError) as ei:
            plan.spectrum(pos, echo)
        assert ei.value.status == sar.SAR_ERR_UNSUPPORTED
        spec = torch_cuda.zeros((sc.grid.ny, sc.grid.nx, len(sc.freq)), dtype=torch_cuda.complex64, device="cuda")
        with pytest.raises(sar.SarError) as ei:
            plan.image_from_spectrum(spec)
        assert ei.value.status == sar.SAR_ERR_UNSUPPORTED
    finally:
        plan.close()


def test_slab_plan_served_equals_plain(torch_cuda):
    # a depth-slab plan and a single-depth one submitted together to a server
    from paper_2305_02064_amd import sar
    scans = [depth_pair_scan(), config1_scan(0)]
    plans = [_plan(scans[0], n_slabs=4), _plan(scans[1])]
    dev = [to_device(sc) for sc in scans]
    srv = sar.Server(4 << 30)
    try:
        refs = [p.reconstruct(d[0], d[1]).clone() for p, d in zip(plans, dev)]
        imgs = [p.new_image() for p in plans]
        # the server runs on its own streams: finish the plain calls first (a
        # buffer they freed may back one of the served images)
        torch_cuda.cuda.synchronize()
        tickets = [srv.submit(p, d[0], d[1], img) for p, d, img in zip(plans, dev, imgs)]
        for t in tickets:
            srv.wait(t)
        for k, (img, ref) in enumerate(zip(imgs, refs)):
            assert rel_l2(img.cpu().numpy(), ref.cpu().numpy()) <= 1e-6, k
    finally:
        srv.close()
        for p in plans:
            p.close()


def _tilted_depth_pair():
    import dataclasses
    sc = depth_pair_scan()
    rng = np.random.default_rng(3)
    pos = sc.pos.copy()
    pos[:, 2] = rng.uniform(-0.015, 0.015, len(pos))
    echo = synth_echo_numpy(pos, sc.tx_xy, sc.rx_xy, sc.freq, sc.targets, sc.amps)
    return dataclasses.replace(sc, pos=pos, echo=echo)


@pytest.mark.parametrize("n_slabs", [0, 4])
def test_amplitude_half_matches_oracle(torch_cuda, n_slabs):
    from paper_2305_02064_amd import sar
    sc = _tilted_depth_pair()
    pos, echo, _ = to_device(sc)
    plan = _plan(sc, n_slabs=n_slabs, flags=sar.SAR_AMPLITUDE)
    try:
        img = plan.reconstruct(pos, echo).cpu().numpy()
    finally:
        plan.close()
    if n_slabs:
        ref = oracle.reconstruct_slabs(sc.pos, sc.tx_xy, sc.rx_xy, sc.freq, sc.echo, sc.grid, n_slabs,
                                       amplitude=True)
        phase_only = oracle.reconstruct_slabs(sc.pos, sc.tx_xy, sc.rx_xy, sc.freq, sc.echo, sc.grid, n_slabs)
    else:
        ref = oracle.reconstruct_direct(sc.pos, sc.tx_xy, sc.rx_xy, sc.freq, sc.echo, sc.grid, amplitude=True)
        phase_only = oracle.reconstruct_direct(sc.pos, sc.tx_xy, sc.rx_xy, sc.freq, sc.echo, sc.grid)
    err = rel_l2(img, ref)
    print(f"tilted depth-pair scene, amplitude half, {n_slabs} slabs: rel-L2 {err:.3e} "
          f"(phase-only image differs by {rel_l2(phase_only, ref):.3e})")
    assert err <= 1e-3
    assert peak_ok(img, ref)
    assert rel_l2(phase_only, ref) > 1e-2
