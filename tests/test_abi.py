"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad descriptors before touching a device."""

import ctypes
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2305_02064_amd", "libsar.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libsar.so not built")


def _sar():
    from paper_2305_02064_amd import sar
    return sar


def test_exports_every_declared_symbol():
    sar = _sar()
    names = sar.header_symbols()
    assert {"sar_plan_create", "sar_reconstruct", "sar_spectrum", "sar_image_from_spectrum",
            "sar_plan_destroy", "sar_last_error"} <= set(names)
    lib = ctypes.CDLL(sar.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_error_string():
    sar = _sar()
    assert "gfx950" in sar.sar_version()
    assert isinstance(sar.sar_last_error(), str)


def _desc_kwargs(**over):
    from sarsynth import awr1443_layout, sweep
    tx, rx = awr1443_layout()
    kw = dict(tx_xy=tx, rx_xy=rx, freq_hz=sweep(16), nx=32, ny=32, nz=16, x0=-0.1, y0=-0.1, z0=0.2,
              dx=0.2 / 32, dy=0.2 / 32, dz=0.0125, z_ref=0.0, z_focus=0.3, max_pos=100)
    kw.update(over)
    return kw


@pytest.mark.parametrize("bad,needle", [
    (dict(nx=28), "products of 2, 3 and 5"),
    (dict(ny=4), "products of 2, 3 and 5"),
    (dict(nx=4096), "products of 2, 3 and 5"),
    (dict(nz=3), "nz"),
    (dict(freq_hz=np.array([78e9, 77e9])), "increasing"),
    (dict(freq_hz=np.array([77e9, np.nan])), "finite"),
    (dict(dx=0.0), "pitch"),
    (dict(z_focus=-0.3), "z_focus"),
    (dict(z0=-0.1), "image volume"),
    (dict(max_pos=-1), "max_pos"),
    (dict(max_pos=2 ** 30), "2^31"),
    (dict(kernel_width=9), "kernel_width"),
    (dict(tol=0.5), "tol"),
    (dict(flags=0x80), "flag"),
    (dict(echo_type=7), "echo type"),
    (dict(n_slabs=3), "n_slabs"),
    (dict(n_slabs=32), "n_slabs"),
    (dict(n_slabs=-2), "n_slabs"),
])
def test_descriptor_validation(bad, needle):
    sar = _sar()
    with pytest.raises(sar.SarError) as ei:
        sar.sar_plan_create(**_desc_kwargs(**bad))
    assert ei.value.status == sar.SAR_ERR_INVALID
    assert needle in str(ei.value)


@pytest.mark.parametrize("bad", [dict(kernel_width=6), dict(echo_type=1)])
def test_fp32_args_diagnostic_limits(bad):
    sar = _sar()
    with pytest.raises(sar.SarError) as ei:
        sar.sar_plan_create(**_desc_kwargs(flags=sar.SAR_FP32_ARGS, **bad))
    assert ei.value.status == sar.SAR_ERR_UNSUPPORTED
    assert "SAR_FP32_ARGS" in str(ei.value)


@pytest.mark.parametrize("up", [1.2, 4.5])
def test_upsample_out_of_range_is_unsupported(up):
    sar = _sar()
    with pytest.raises(sar.SarError) as ei:
        sar.sar_plan_create(**_desc_kwargs(upsample=up))
    assert ei.value.status == sar.SAR_ERR_UNSUPPORTED
    assert "1.25" in str(ei.value)


def test_null_arguments():
    sar = _sar()
    lib = sar.library()
    b = ctypes.c_size_t()
    assert lib.sar_plan_workspace_bytes(None, 0, ctypes.byref(b)) == sar.SAR_ERR_INVALID
    assert lib.sar_reconstruct(None, None, 0, None, 1.0, None, None, None) == sar.SAR_ERR_INVALID
    assert lib.sar_plan_create(None, 0, None) == sar.SAR_ERR_INVALID
    assert lib.sar_plan_destroy(None) == sar.SAR_OK


def test_server_null_and_budget_arguments():
    # argument checks that return before any device call
    sar = _sar()
    lib = sar.library()
    h = ctypes.c_void_p()
    assert lib.sar_server_create(0, 1 << 20, None) == sar.SAR_ERR_INVALID
    assert lib.sar_server_create(0, 16, ctypes.byref(h)) == sar.SAR_ERR_INVALID
    assert "budget" in sar.sar_last_error()
    t = ctypes.c_uint64()
    assert lib.sar_submit(None, None, None, 0, None, 1, 1.0, None, ctypes.byref(t)) == sar.SAR_ERR_INVALID
    done = ctypes.c_int()
    assert lib.sar_poll(None, 1, ctypes.byref(done), None) == sar.SAR_ERR_INVALID
    assert lib.sar_server_destroy(None) == sar.SAR_OK


def test_batch_null_arguments():
    sar = _sar()
    lib = sar.library()
    h = ctypes.c_void_p()
    assert lib.sar_batch_create(None, 0, 0, ctypes.byref(h)) == sar.SAR_ERR_INVALID
    arr = (ctypes.c_void_p * 1)(None)
    assert lib.sar_batch_create(arr, 1, 0, ctypes.byref(h)) == sar.SAR_ERR_INVALID
    assert "NULL" in sar.sar_last_error()
    assert lib.sar_batch_create(arr, 1, 0, None) == sar.SAR_ERR_INVALID
    b = ctypes.c_size_t()
    assert lib.sar_batch_workspace_bytes(None, ctypes.byref(b)) == sar.SAR_ERR_INVALID
    assert lib.sar_batch_reconstruct(None, None, None, None, None, None, None, None) == sar.SAR_ERR_INVALID
    assert lib.sar_batch_destroy(None) == sar.SAR_OK


def test_grid_tile_arguments():
    sar = _sar()
    lib = sar.library()
    assert lib.sar_plan_set_grid_tile(None, 0) == sar.SAR_ERR_INVALID
    t = ctypes.c_int32()
    assert lib.sar_plan_autotune(None, None, 0, None, 1.0, None, None, ctypes.byref(t)) == sar.SAR_ERR_INVALID


def test_oversampled_grid_beyond_longest_transform_is_refused_at_plan_creation():
    # 2048 voxels at upsample 3 asks for 6144+ cells along x: refused before any
    # kernel is queued (the lateral transforms stop at 4096 points)
    sar = _sar()
    with pytest.raises(sar.SarError) as ei:
        sar.sar_plan_create(**_desc_kwargs(nx=2048, upsample=3.0))
    assert ei.value.status == sar.SAR_ERR_UNSUPPORTED
    assert "4096" in str(ei.value)


def _fake_info(sar, **over):
    info = sar.sar_plan_info()
    vals = dict(nx=8, ny=16, nz=4, n_freq=5, n_pair=2, echo_type=sar.SAR_ECHO_C64, max_pos=10)
    vals.update(over)
    for k, v in vals.items():
        setattr(info, k, v)
    return info


@pytest.mark.parametrize("case", ["pos_flat", "pos_rows", "pos_dtype", "echo_size", "echo_dtype",
                                  "half_as_c64", "c64_as_half"])
def test_wrappers_check_scan_inputs_against_the_plan(case):
    # the C ABI receives raw pointers and cannot check buffer sizes: the Python
    # binding compares every scan input with the plan before any pointer is
    # passed on (CPU tensors here; the check runs before the device check)
    import torch
    sar = _sar()
    n = 3
    pos = torch.zeros((n, 3), dtype=torch.float64)
    echo = torch.zeros((n, 2, 5), dtype=torch.complex64)
    info = _fake_info(sar)
    if case == "pos_flat":
        pos = pos.reshape(-1)
    elif case == "pos_rows":
        pos = torch.zeros((n - 1, 3), dtype=torch.float64)
    elif case == "pos_dtype":
        pos = pos.float()
    elif case == "echo_size":
        echo = torch.zeros((n, 2, 4), dtype=torch.complex64)
    elif case == "echo_dtype":
        echo = echo.to(torch.complex128)
    elif case == "half_as_c64":
        echo = torch.zeros((n, 2, 5, 2), dtype=torch.float16)
    elif case == "c64_as_half":
        info = _fake_info(sar, echo_type=sar.SAR_ECHO_F16X2)
    with pytest.raises(ValueError):
        sar._check_scan(info, pos, n, echo)


def test_wrappers_accept_matching_inputs_and_check_outputs(monkeypatch):
    import torch
    sar = _sar()
    info = _fake_info(sar)
    sar._check_scan(info, torch.zeros((3, 3), dtype=torch.float64), 3, torch.zeros((3, 2, 5), dtype=torch.complex64))
    sar._check_scan(info, torch.zeros((3, 3), dtype=torch.float64), 3, torch.zeros((3, 2, 5, 2), dtype=torch.float32))
    h = _fake_info(sar, echo_type=sar.SAR_ECHO_F16X2)
    sar._check_scan(h, torch.zeros((3, 3), dtype=torch.float64), 3, torch.zeros((3, 2, 5, 2), dtype=torch.float16))
    # larger buffers than the call uses are fine (the first n_pos shots are read)
    sar._check_scan(info, torch.zeros((5, 3), dtype=torch.float64), 3, torch.zeros((5, 2, 5), dtype=torch.complex64))
    assert sar._image_shape(info) == (8, 16, 4) and sar._spectrum_shape(info) == (16, 8, 5)
    # a wrong image shape is caught before the library call
    calls = []
    monkeypatch.setattr(sar, "_info", lambda plan: info)
    monkeypatch.setattr(sar, "library", lambda: calls.append(1))
    with pytest.raises(ValueError):
        sar.sar_reconstruct(None, torch.zeros((3, 3), dtype=torch.float64), 3,
                            torch.zeros((3, 2, 5), dtype=torch.complex64), 1.0,
                            torch.zeros((8, 16, 5), dtype=torch.complex64), torch.zeros(16, dtype=torch.uint8))
    assert not calls

