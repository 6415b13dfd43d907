"""GPU tests of fused batches of uneven scans (sar_batch_* through the C ABI).

A batch runs every item's pipeline inside shared fused launches (and, by
default, replays one captured HIP graph), so each item's image must equal
the plain per-scan image of the same inputs (the kernels and their order per
scan are the same: relative L2 <= 1e-6), on every replay, with new inputs and
with fewer shots than the plan's maximum, and with plain work between
replays.  A batched tiny scan must match the FP64 oracle, and scans of the
uneven batch with their scene echoes must match it on sampled spectrum entries.
"""

import numpy as np
import pytest

import oracle
from sarsynth import config1_scan, config4_scan
from tests.sar_testutil import make_plan, peak_ok, rel_l2, to_device

pytestmark = pytest.mark.gpu

SAME_TOL = 1e-6


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _random_echo(torch, shape, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    return torch.complex(torch.randn(shape, generator=g, device="cuda"), torch.randn(shape, generator=g, device="cuda"))


@pytest.fixture(scope="module")
def items(torch_cuda):
    """Uneven scans (image sides 128 and 256, 64-256 frequencies) plus the tiny scan."""
    from paper_2305_02064_amd import sar
    out = []
    for seed in (4, 5, 8, 11, 1):
        sc = config4_scan(seed, with_echo=False)
        pos = torch_cuda.from_numpy(np.ascontiguousarray(sc.pos)).cuda()
        echo = _random_echo(torch_cuda, (sc.n_pos, sc.n_pair, sc.n_freq), 500 + seed)
        out.append((sc, sar.Plan(sc.tx_xy, sc.rx_xy, sc.freq, sc.grid, sc.n_pos), pos, echo))
    tiny = config1_scan(0)
    pos, echo, _ = to_device(tiny)
    out.append((tiny, make_plan(tiny), pos, echo))
    return out


def _plain(items_, pos=None, echo=None):
    imgs = []
    for k, (sc, plan, p0, e0) in enumerate(items_):
        imgs.append(plan.reconstruct(p0 if pos is None else pos[k], e0 if echo is None else echo[k]).clone())
    return imgs


@pytest.mark.parametrize("graph", [True, False])
def test_batch_equals_plain(torch_cuda, items, graph):
    from paper_2305_02064_amd import sar
    refs = _plain(items)
    b = sar.Batch([it[1] for it in items], graph=graph)
    try:
        imgs = b.reconstruct([it[2] for it in items], [it[3] for it in items])
        torch_cuda.cuda.synchronize()
    finally:
        b.close()
    for k, (img, ref) in enumerate(zip(imgs, refs)):
        err = rel_l2(img.cpu().numpy(), ref.cpu().numpy())
        assert err <= SAME_TOL, (k, err)
    print(f"batch ({'graph' if graph else 'direct'}) of {len(items)} uneven scans equals plain "
          f"({sum(int(torch_cuda.equal(a, r)) for a, r in zip(imgs, refs))} bit-identical)")


def test_graph_replays_with_new_inputs(torch_cuda, items):
    # three replays of the captured graph with different echoes, one item with
    # fewer shots than its plan's maximum, plain work in between
    from paper_2305_02064_amd import sar
    b = sar.Batch([it[1] for it in items])
    try:
        for rep in range(3):
            pos = [it[2] for it in items]
            echo = [_random_echo(torch_cuda, tuple(it[3].shape), 900 + 10 * rep + k) for k, it in enumerate(items)]
            if rep == 1:
                cut = items[0][2].shape[0] // 3
                pos[0] = pos[0][:cut].contiguous()
                echo[0] = echo[0][:cut].contiguous()
            imgs = b.reconstruct(pos, echo)
            refs = _plain(items, pos, echo)   # eager work between the replays
            torch_cuda.cuda.synchronize()
            for k, (img, ref) in enumerate(zip(imgs, refs)):
                err = rel_l2(img.cpu().numpy(), ref.cpu().numpy())
                assert err <= SAME_TOL, (rep, k, err)
    finally:
        b.close()


def test_batched_tiny_scan_matches_oracle(torch_cuda, items):
    from paper_2305_02064_amd import sar
    tiny = items[-1][0]
    ref = oracle.reconstruct_direct(tiny.pos, tiny.tx_xy, tiny.rx_xy, tiny.freq, tiny.echo, tiny.grid)
    b = sar.Batch([it[1] for it in items])
    try:
        img = b.reconstruct([it[2] for it in items], [it[3] for it in items])[-1].cpu().numpy()
    finally:
        b.close()
    err = rel_l2(img, ref)
    print(f"batched tiny scan rel-L2 {err:.3e}")
    assert err <= 1e-3
    assert peak_ok(img, ref)


def test_batch_rejects_bad_items(torch_cuda, items):
    from paper_2305_02064_amd import sar
    b = sar.Batch([it[1] for it in items[:2]])
    try:
        sc, plan, pos, echo = items[0]
        big_pos = torch_cuda.cat([pos, pos[:1]])
        big_echo = torch_cuda.cat([echo, echo[:1]])
        with pytest.raises(sar.SarError) as ei:
            b.reconstruct([big_pos, items[1][2]], [big_echo, items[1][3]])
        assert ei.value.status == sar.SAR_ERR_INVALID
        assert "item 0" in str(ei.value)
        with pytest.raises(ValueError):
            b.reconstruct([pos], [echo])
    finally:
        b.close()


def test_uneven_scans_match_oracle_on_sampled_entries(torch_cuda):
    # scans of the uneven batch with their scene echoes, run as one fused
    # batch; each scan's spectrum at 96 sampled (k_x, k_y, f) entries is an
    # exact sum over all of its virtual samples in the oracle
    from paper_2305_02064_amd import sar
    scans = [config4_scan(seed, device=torch_cuda.device("cuda", 0)) for seed in (5, 9, 11)]
    plans = [sar.Plan(sc.tx_xy, sc.rx_xy, sc.freq, sc.grid, sc.n_pos) for sc in scans]
    pos = [torch_cuda.from_numpy(np.ascontiguousarray(sc.pos)).cuda() for sc in scans]
    specs = [p.spectrum(q, sc.echo).cpu().numpy() for p, q, sc in zip(plans, pos, scans)]
    imgs_plain = [p.reconstruct(q, sc.echo) for p, q, sc in zip(plans, pos, scans)]
    b = sar.Batch(plans)
    try:
        imgs = b.reconstruct(pos, [sc.echo for sc in scans])
        torch_cuda.cuda.synchronize()
    finally:
        b.close()
    for k, sc in enumerate(scans):
        assert rel_l2(imgs[k].cpu().numpy(), imgs_plain[k].cpu().numpy()) <= SAME_TOL
        g = sc.grid
        rng = np.random.default_rng(60 + k)
        ne = 96
        qi, pi, fi = rng.integers(0, g.ny, ne), rng.integers(0, g.nx, ne), rng.integers(0, sc.n_freq, ne)
        kw = oracle.wavenumber(sc.freq)
        xv, yv, dxx, dyy, dzz = oracle.virtual_samples(sc.pos, sc.tx_xy, sc.rx_xy, g.z_ref)
        beta = oracle.residual_path(dxx, dyy, dzz, g.z_ref, g.z_focus).ravel()
        kx, ky, xc, yc = oracle.mode_axes(g.nx, g.ny, g.x0, g.y0, g.dx, g.dy)
        uf = np.unique(fi)
        e_host = sc.echo[:, :, uf].cpu().numpy().reshape(-1, len(uf))
        shat = oracle.compensate(e_host, kw[uf], beta)
        ref = oracle.nudft2_entries(shat, xv.ravel(), yv.ravel(), kx[pi], ky[qi], np.searchsorted(uf, fi), xc, yc)
        err = rel_l2(specs[k][qi, pi, fi], ref)
        print(f"uneven scan {sc.meta['config']}: sampled spectrum rel-L2 {err:.3e}")
        assert err <= 1e-3
