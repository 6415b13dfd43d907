"""sar_reconstruct_noalloc (the entry point for callers that cannot allocate)
through the C ABI against sar_reconstruct on the same inputs: two calls in a
row, the second with fewer shots, each equal to the plain call's image (same
kernels, same launches, so bit-identical), and a scan too large for the fixed
scratch refused up front."""

import numpy as np
import pytest

from sarsynth import config1_scan, config4_scan
from tests.sar_testutil import make_plan, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _plain(plan, pos, n, echo):
    from paper_2305_02064_amd import sar
    img = plan.new_image()
    sar.sar_reconstruct(plan.handle, pos[:n], n, echo[:n], 1.0, img, plan.ws)
    return img


def test_noalloc_equals_plain_on_two_calls(torch_cuda):
    from paper_2305_02064_amd import sar
    scan = config1_scan(0)
    plan = make_plan(scan)
    pos, echo, _ = to_device(scan)
    for n in (scan.n_pos, scan.n_pos // 3):   # the second call is smaller
        print(f"noalloc: tiny scan, {n} shots", flush=True)
        ref = _plain(plan, pos, n, echo)
        img = plan.new_image()
        img.fill_(float("nan"))
        sar.sar_reconstruct_noalloc(plan.handle, pos[:n].contiguous(), n, echo[:n].contiguous(), 1.0, img)
        torch_cuda.cuda.synchronize()
        a, b = img.cpu().numpy(), ref.cpu().numpy()
        assert np.isfinite(a).all()
        assert np.array_equal(a, b), float(np.abs(a - b).max())


def test_noalloc_other_plan_after_a_larger_one(torch_cuda):
    # a different plan (small uneven-batch scan, random echo) on the same
    # scratch after the tiny scan: still equal to its plain image
    from paper_2305_02064_amd import sar
    sc = None
    for seed in range(64):
        c = config4_scan(seed, with_echo=False)
        plan = sar.Plan(c.tx_xy, c.rx_xy, c.freq, c.grid, c.n_pos)
        need = sar.sar_plan_workspace_bytes(plan.handle, c.n_pos)
        if need <= (64 << 20):
            sc = c
            break
        plan.close()
    assert sc is not None
    print(f"noalloc: uneven-batch scan seed {seed}, {sc.n_pos} shots, {need} bytes", flush=True)
    g = torch_cuda.Generator(device="cuda")
    g.manual_seed(5)
    shape = (sc.n_pos, sc.n_pair, sc.n_freq)
    echo = torch_cuda.complex(torch_cuda.randn(shape, generator=g, device="cuda"),
                              torch_cuda.randn(shape, generator=g, device="cuda"))
    pos = torch_cuda.from_numpy(np.ascontiguousarray(sc.pos)).cuda()
    ref = _plain(plan, pos, sc.n_pos, echo)
    img = plan.new_image()
    sar.sar_reconstruct_noalloc(plan.handle, pos, sc.n_pos, echo, 1.0, img)
    torch_cuda.cuda.synchronize()
    assert torch_cuda.equal(img, ref)


def test_noalloc_refuses_scans_beyond_the_scratch(torch_cuda):
    from paper_2305_02064_amd import sar
    scan = config1_scan(0)
    big = make_plan(scan, max_pos=150000)
    pos = torch_cuda.zeros((150000, 3), dtype=torch_cuda.float64, device="cuda")
    echo = torch_cuda.zeros((150000, scan.n_pair, scan.n_freq), dtype=torch_cuda.complex64, device="cuda")
    img = big.new_image()
    with pytest.raises(sar.SarError) as ei:
        sar.sar_reconstruct_noalloc(big.handle, pos, 150000, echo, 1.0, img)
    assert ei.value.status == sar.SAR_ERR_UNSUPPORTED
    assert "scratch" in str(ei.value)
