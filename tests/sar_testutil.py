"""Helpers shared by the GPU tests: plans from synthetic scans, device copies,
error metrics.  The oracle side never sees anything computed on the GPU."""

import numpy as np


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def peak_index(img):
    return np.unravel_index(int(np.argmax(np.abs(img))), img.shape)


def peak_ok(gpu_img, ref_img, rel_gap=1e-4):
    """Exact peak voxel; if the reference's top two voxels are within rel_gap of
    each other either is accepted (several results are then correct)."""
    a = np.abs(ref_img).ravel()
    order = np.argsort(a)[::-1]
    g = int(np.argmax(np.abs(gpu_img).ravel()))
    if g == order[0]:
        return True
    return g == order[1] and (a[order[0]] - a[order[1]]) <= rel_gap * a[order[0]]


def make_plan(scan, max_pos=None, **kw):
    from paper_2305_02064_amd import sar
    return sar.Plan(scan.tx_xy, scan.rx_xy, scan.freq, scan.grid,
                    scan.n_pos if max_pos is None else max_pos, **kw)


def to_device(scan, half=False):
    import torch
    pos = torch.from_numpy(np.ascontiguousarray(scan.pos, np.float64)).cuda()
    e = scan.echo
    if isinstance(e, torch.Tensor):
        echo = e.contiguous()
    else:
        echo = torch.from_numpy(np.ascontiguousarray(e, np.complex64)).cuda()
    if not half:
        return pos, echo, 1.0
    # FP16 storage with one scale per scan: max |Re|, |Im| mapped to 2^15
    er = torch.view_as_real(echo)
    amax = float(er.abs().max().item())
    scale = amax / 32768.0 if amax > 0 else 1.0
    eh = (er / scale).to(torch.float16).contiguous()
    return pos, eh, scale
