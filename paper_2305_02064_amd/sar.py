"""Thin Python binding of libsar (include/sar.h).

Argument marshalling only: every step of the image formation runs in the HIP
kernels of libsar.so.  PyTorch provides device memory and streams; tensors are
passed to the library as raw device pointers.  Importing this module loads the
in-tree libsar.so and fails loudly when it is missing (there is no fallback).
"""

from __future__ import annotations

import ctypes
import os
import re

import torch  # noqa: F401  (loads the HIP runtime the library shares with torch)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsar.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "sar.h")

SAR_OK = 0
SAR_ERR_INVALID = 1
SAR_ERR_NOMEM = 2
SAR_ERR_DEVICE = 3
SAR_ERR_BUSY = 4
SAR_ERR_NOT_FOUND = 5
SAR_ERR_UNSUPPORTED = 6
STATUS_NAMES = {0: "SAR_OK", 1: "SAR_ERR_INVALID", 2: "SAR_ERR_NOMEM", 3: "SAR_ERR_DEVICE", 4: "SAR_ERR_BUSY",
                5: "SAR_ERR_NOT_FOUND", 6: "SAR_ERR_UNSUPPORTED"}

SAR_ECHO_C64 = 0
SAR_ECHO_F16X2 = 1
SAR_NO_COMPENSATION = 0x1
SAR_FP32_ARGS = 0x2
SAR_STOLT_DCF = 0x4
SAR_AMPLITUDE = 0x8
SAR_BATCH_NO_GRAPH = 0x1

STAGES = ("geometry+sort", "gridding", "fft_x", "fft_y", "stolt", "ifft_y", "ifft_x")


class SarError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class sar_plan_desc(ctypes.Structure):
    _fields_ = [
        ("n_tx", ctypes.c_int32), ("n_rx", ctypes.c_int32),
        ("tx_xy", ctypes.POINTER(ctypes.c_double)), ("rx_xy", ctypes.POINTER(ctypes.c_double)),
        ("n_freq", ctypes.c_int32), ("freq_hz", ctypes.POINTER(ctypes.c_double)),
        ("z_ref", ctypes.c_double), ("z_focus", ctypes.c_double),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("z0", ctypes.c_double),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("max_pos", ctypes.c_int64),
        ("echo_type", ctypes.c_int32),
        ("tol", ctypes.c_double), ("upsample", ctypes.c_double),
        ("kernel_width", ctypes.c_int32), ("flags", ctypes.c_uint32),
        ("n_slabs", ctypes.c_int32),
    ]


class sar_plan_info(ctypes.Structure):
    _fields_ = [
        ("mx", ctypes.c_int32), ("my", ctypes.c_int32), ("width", ctypes.c_int32),
        ("kb_beta", ctypes.c_double),
        ("mz", ctypes.c_int32), ("width_z", ctypes.c_int32),
        ("es_beta_z", ctypes.c_double),
        ("n_pair", ctypes.c_int32), ("n_stages", ctypes.c_int32),
        ("workspace_bytes_max", ctypes.c_size_t),
        ("grid_tile", ctypes.c_int32), ("grid_tile_x", ctypes.c_int32), ("grid_tile_y", ctypes.c_int32),
        ("grid_freqs_per_lane", ctypes.c_int32),
        ("n_slabs", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("n_freq", ctypes.c_int32), ("echo_type", ctypes.c_int32), ("flags", ctypes.c_uint32),
        ("max_pos", ctypes.c_int64),
        ("sigma_x", ctypes.c_double), ("sigma_y", ctypes.c_double),
    ]


_lib = None


def library():
    """Load libsar.so (once).  Raises ImportError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libsar.so not found at {LIB_PATH}; build it with "
                          f"`python -m paper_2305_02064_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    sig = {
        "sar_plan_create": ([ctypes.POINTER(sar_plan_desc), ctypes.c_int, ctypes.POINTER(vp)], i32),
        "sar_plan_destroy": ([vp], i32),
        "sar_plan_workspace_bytes": ([vp, i64, ctypes.POINTER(ctypes.c_size_t)], i32),
        "sar_plan_get_info": ([vp, ctypes.POINTER(sar_plan_info)], i32),
        "sar_reconstruct": ([vp, vp, i64, vp, f32, vp, vp, vp], i32),
        "sar_spectrum": ([vp, vp, i64, vp, f32, vp, vp, vp], i32),
        "sar_reconstruct_noalloc": ([vp, vp, i64, vp, f32, vp, vp], i32),
        "sar_image_from_spectrum": ([vp, vp, vp, vp, vp], i32),
        "sar_plan_set_timing": ([vp, ctypes.c_int], i32),
        "sar_plan_autotune": ([vp, vp, i64, vp, f32, vp, vp, ctypes.POINTER(i32)], i32),
        "sar_plan_set_grid_tile": ([vp, i32], i32),
        "sar_backproject": ([vp, vp, i64, vp, f32, vp, vp], i32),
        "sar_plan_stage_times": ([vp, ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(i64)], i32),
        "sar_server_create": ([ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(vp)], i32),
        "sar_submit": ([vp, vp, vp, i64, vp, ctypes.c_int, f32, vp, ctypes.POINTER(ctypes.c_uint64)], i32),
        "sar_poll": ([vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)], i32),
        "sar_server_destroy": ([vp], i32),
        "sar_batch_create": ([ctypes.POINTER(vp), i32, ctypes.c_uint32, ctypes.POINTER(vp)], i32),
        "sar_batch_workspace_bytes": ([vp, ctypes.POINTER(ctypes.c_size_t)], i32),
        "sar_batch_reconstruct": ([vp, ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.POINTER(vp),
                                   ctypes.POINTER(f32), ctypes.POINTER(vp), vp, vp], i32),
        "sar_batch_destroy": ([vp], i32),
        "sar_last_error": ([], ctypes.c_char_p),
        "sar_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def header_symbols():
    """Names of the functions include/sar.h declares."""
    with open(HEADER_PATH) as f:
        txt = f.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(sar_\w+)\s*\(", txt, flags=re.M)))


def _check(status):
    if status != SAR_OK:
        raise SarError(status, library().sar_last_error().decode())


def sar_last_error():
    return library().sar_last_error().decode()


def sar_version():
    return library().sar_version().decode()


def _dptr(t, name, dtype=None, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _info(plan):
    info = sar_plan_info()
    _check(library().sar_plan_get_info(plan, ctypes.byref(info)))
    return info


def _check_scan(info, pos, n_pos, echo):
    """Shapes and types of one scan's inputs against the plan, before any
    pointer reaches the library (which cannot check buffer sizes itself)."""
    n_pos = int(n_pos)
    if not isinstance(pos, torch.Tensor) or not isinstance(echo, torch.Tensor):
        raise TypeError("pos and echo must be torch tensors")
    # buffers may hold more shots than the call uses (the library reads the
    # first n_pos), never fewer
    if pos.dtype != torch.float64 or pos.dim() != 2 or pos.shape[1] != 3 or pos.shape[0] < n_pos:
        raise ValueError(f"pos must be float64 of shape (>= {n_pos}, 3), got {pos.dtype} {tuple(pos.shape)}")
    n_val = n_pos * info.n_pair * info.n_freq
    if info.echo_type == SAR_ECHO_C64:
        ok = (echo.dtype == torch.complex64 and echo.numel() >= n_val) or \
             (echo.dtype == torch.float32 and echo.numel() >= 2 * n_val)
        want = f"complex64 with >= {n_val} values (or float32 with >= {2 * n_val})"
    else:
        ok = echo.dtype == torch.float16 and echo.numel() >= 2 * n_val
        want = f"float16 with >= {2 * n_val} values (real/imaginary pairs)"
    if not ok:
        raise ValueError(f"echo must be {want} for this plan ({n_pos} shots x {info.n_pair} pairs x "
                         f"{info.n_freq} frequencies), got {echo.dtype} with {echo.numel()}")


def _image_shape(info):
    return (info.nx, info.ny, info.nz)


def _spectrum_shape(info):
    return (info.ny, info.nx, info.n_freq)


def _check_workspace(plan, n_pos, workspace):
    need = sar_plan_workspace_bytes(plan, n_pos)
    if workspace.numel() * workspace.element_size() < need:
        raise ValueError(f"workspace holds {workspace.numel() * workspace.element_size()} bytes; "
                         f"the scan needs {need}")


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def sar_plan_create(tx_xy, rx_xy, freq_hz, nx, ny, nz, x0, y0, z0, dx, dy, dz, z_ref, z_focus, max_pos,
                    echo_type=SAR_ECHO_C64, tol=0.0, upsample=0.0, kernel_width=0, flags=0, n_slabs=0, device=0):
    """Create a plan (see sar_plan_create in include/sar.h); returns an opaque handle."""
    import numpy as np
    lib = library()
    tx = np.ascontiguousarray(tx_xy, dtype=np.float64).reshape(-1, 2)
    rx = np.ascontiguousarray(rx_xy, dtype=np.float64).reshape(-1, 2)
    fr = np.ascontiguousarray(freq_hz, dtype=np.float64).ravel()
    dp = ctypes.POINTER(ctypes.c_double)
    d = sar_plan_desc(
        n_tx=len(tx), n_rx=len(rx), tx_xy=tx.ctypes.data_as(dp), rx_xy=rx.ctypes.data_as(dp),
        n_freq=len(fr), freq_hz=fr.ctypes.data_as(dp), z_ref=z_ref, z_focus=z_focus,
        nx=nx, ny=ny, nz=nz, x0=x0, y0=y0, z0=z0, dx=dx, dy=dy, dz=dz, max_pos=max_pos,
        echo_type=echo_type, tol=tol, upsample=upsample, kernel_width=kernel_width, flags=flags, n_slabs=n_slabs)
    h = ctypes.c_void_p()
    _check(lib.sar_plan_create(ctypes.byref(d), int(device), ctypes.byref(h)))
    return h


def sar_plan_destroy(plan):
    _check(library().sar_plan_destroy(plan))


def sar_plan_workspace_bytes(plan, n_pos):
    b = ctypes.c_size_t()
    _check(library().sar_plan_workspace_bytes(plan, int(n_pos), ctypes.byref(b)))
    return int(b.value)


def sar_plan_get_info(plan):
    info = sar_plan_info()
    _check(library().sar_plan_get_info(plan, ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in sar_plan_info._fields_}


def sar_reconstruct(plan, pos, n_pos, echo, echo_scale, image, workspace, stream=None):
    info = _info(plan)
    _check_scan(info, pos, n_pos, echo)
    args = (_dptr(pos, "pos", torch.float64), int(n_pos), _dptr(echo, "echo"), float(echo_scale),
            _dptr(image, "image", torch.complex64, _image_shape(info)), _dptr(workspace, "workspace"))
    _check_workspace(plan, n_pos, workspace)
    _check(library().sar_reconstruct(plan, *args, _stream(stream)))


def sar_reconstruct_noalloc(plan, pos, n_pos, echo, echo_scale, image, stream=None):
    """sar_reconstruct with the library's fixed scratch as workspace (no allocation)."""
    info = _info(plan)
    _check_scan(info, pos, n_pos, echo)
    args = (_dptr(pos, "pos", torch.float64), int(n_pos), _dptr(echo, "echo"), float(echo_scale),
            _dptr(image, "image", torch.complex64, _image_shape(info)))
    _check(library().sar_reconstruct_noalloc(plan, *args, _stream(stream)))


def sar_spectrum(plan, pos, n_pos, echo, echo_scale, spectrum, workspace, stream=None):
    info = _info(plan)
    _check_scan(info, pos, n_pos, echo)
    args = (_dptr(pos, "pos", torch.float64), int(n_pos), _dptr(echo, "echo"), float(echo_scale),
            _dptr(spectrum, "spectrum", torch.complex64, _spectrum_shape(info)), _dptr(workspace, "workspace"))
    _check_workspace(plan, n_pos, workspace)
    _check(library().sar_spectrum(plan, *args, _stream(stream)))


def sar_image_from_spectrum(plan, spectrum, image, workspace, stream=None):
    info = _info(plan)
    args = (_dptr(spectrum, "spectrum", torch.complex64, _spectrum_shape(info)),
            _dptr(image, "image", torch.complex64, _image_shape(info)), _dptr(workspace, "workspace"))
    _check_workspace(plan, 0, workspace)
    _check(library().sar_image_from_spectrum(plan, *args, _stream(stream)))


def sar_plan_set_timing(plan, enable):
    _check(library().sar_plan_set_timing(plan, 1 if enable else 0))


def sar_plan_stage_times(plan):
    """Summed per-stage milliseconds over the recorded calls, and their count."""
    ms = (ctypes.c_double * len(STAGES))()
    n = ctypes.c_int64()
    _check(library().sar_plan_stage_times(plan, ms, len(STAGES), ctypes.byref(n)))
    return dict(zip(STAGES, list(ms))), int(n.value)


def _ptr(t, name, dtype=None):
    """Raw pointer of a contiguous host or device tensor."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def sar_server_create(device, hbm_budget_bytes):
    h = ctypes.c_void_p()
    _check(library().sar_server_create(int(device), int(hbm_budget_bytes), ctypes.byref(h)))
    return h


def sar_submit(server, plan, pos, n_pos, echo, echo_scale, image):
    """Queue one scan; pos and echo are both device tensors or both host tensors."""
    if pos.is_cuda != echo.is_cuda:
        raise ValueError("pos and echo must both be on the device or both on the host")
    info = _info(plan)
    _check_scan(info, pos, n_pos, echo)
    _dptr(image, "image", torch.complex64, _image_shape(info))
    t = ctypes.c_uint64()
    _check(library().sar_submit(server, plan, _ptr(pos, "pos", torch.float64), int(n_pos), _ptr(echo, "echo"),
                                1 if echo.is_cuda else 0, float(echo_scale),
                                _dptr(image, "image", torch.complex64), ctypes.byref(t)))
    return int(t.value)


def sar_poll(server, ticket):
    """(done, latency_s); raises SarError if the scan failed."""
    done = ctypes.c_int()
    lat = ctypes.c_double()
    _check(library().sar_poll(server, ctypes.c_uint64(ticket), ctypes.byref(done), ctypes.byref(lat)))
    return bool(done.value), (float(lat.value) if done.value else None)


def sar_server_destroy(server):
    _check(library().sar_server_destroy(server))


class Batch:
    """A fused batch (sar_batch_*): one plan per item; reconstruct() images
    every item in one fused launch per pipeline step (a captured HIP graph
    unless graph=False)."""

    def __init__(self, plans, graph=True):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(library().sar_batch_create(arr, len(self.plans), 0 if graph else SAR_BATCH_NO_GRAPH,
                                          ctypes.byref(h)))
        self.handle = h
        b = ctypes.c_size_t()
        _check(library().sar_batch_workspace_bytes(h, ctypes.byref(b)))
        nbytes = max(int(b.value), 256)
        dev = self.plans[0].device
        self._ws_buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        off = (-self._ws_buf.data_ptr()) % 256
        self.ws = self._ws_buf[off:off + nbytes]

    def reconstruct(self, pos, echo, images=None, echo_scale=None, stream=None):
        n = len(self.plans)
        if len(pos) != n or len(echo) != n:
            raise ValueError(f"need {n} position and echo tensors")
        images = [p.new_image() for p in self.plans] if images is None else images
        if len(images) != n:
            raise ValueError(f"need {n} images")
        for p, ps, e, im in zip(self.plans, pos, echo, images):
            info = _info(p.handle)
            _check_scan(info, ps, ps.shape[0], e)
            _dptr(ps, "pos", torch.float64)
            _dptr(e, "echo")
            _dptr(im, "image", torch.complex64, _image_shape(info))
        vp = ctypes.c_void_p
        P = (vp * n)(*[_dptr(t, "pos", torch.float64).value for t in pos])
        N = (ctypes.c_int64 * n)(*[t.shape[0] for t in pos])
        E = (vp * n)(*[_dptr(t, "echo").value for t in echo])
        S = (ctypes.c_float * n)(*([1.0] * n if echo_scale is None else [float(x) for x in echo_scale]))
        I = (vp * n)(*[_dptr(t, "image", torch.complex64).value for t in images])
        _check(library().sar_batch_reconstruct(self.handle, P, N, E, S, I, _dptr(self.ws, "workspace"),
                                               _stream(stream)))
        return images

    def close(self):
        if self.handle is not None:
            library().sar_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """A serving loop (sar_server_*): scans are submitted, overlap on the
    device under an HBM budget, and are collected by polling.  The buffers of
    a submitted scan are kept referenced here until it is collected."""

    def __init__(self, hbm_budget_bytes, device=0):
        self.device = torch.device("cuda", device)
        self.handle = sar_server_create(device, hbm_budget_bytes)
        self._held = {}

    def submit(self, plan, pos, echo, image=None, echo_scale=1.0):
        image = plan.new_image() if image is None else image
        ticket = sar_submit(self.handle, plan.handle, pos, pos.shape[0], echo, echo_scale, image)
        # the plan too must outlive the request: keep the Plan object (whose
        # finaliser destroys the handle) referenced until the scan is collected
        self._held[ticket] = (pos, echo, image, plan)
        return ticket

    def poll(self, ticket):
        """(done, latency_s, image); image is None until done."""
        try:
            done, lat = sar_poll(self.handle, ticket)
        except SarError:
            self._held.pop(ticket, None)
            raise
        if not done:
            return False, None, None
        return True, lat, self._held.pop(ticket)[2]

    def wait(self, ticket, timeout=60.0, spin=50e-6):
        """Poll until the scan is done; returns (latency_s, image)."""
        import time
        t_end = time.perf_counter() + timeout
        while True:
            done, lat, img = self.poll(ticket)
            if done:
                return lat, img
            if time.perf_counter() > t_end:
                raise TimeoutError(f"scan {ticket} not done after {timeout} s")
            time.sleep(spin)

    def close(self):
        if self.handle is not None:
            sar_server_destroy(self.handle)
            self.handle = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Owns a plan handle plus (unless workspace=False) a device workspace
    sized for max_pos shots."""

    def __init__(self, tx_xy, rx_xy, freq_hz, grid, max_pos, device=0, workspace=True, **kw):
        self.grid = grid
        self.device = torch.device("cuda", device)
        self.n_pair = len(tx_xy) * len(rx_xy)
        self.n_freq = len(freq_hz)
        self.handle = sar_plan_create(tx_xy, rx_xy, freq_hz, grid.nx, grid.ny, grid.nz, grid.x0, grid.y0,
                                      grid.z0, grid.dx, grid.dy, grid.dz, grid.z_ref, grid.z_focus, max_pos,
                                      device=device, **kw)
        self.info = sar_plan_get_info(self.handle)
        self.max_pos = max_pos
        self.workspace = self.ws = None
        if workspace:
            nbytes = max(self.info["workspace_bytes_max"], 256)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-self.workspace.data_ptr()) % 256
            self.ws = self.workspace[off:off + nbytes]

    def new_image(self):
        g = self.grid
        return torch.empty((g.nx, g.ny, g.nz), dtype=torch.complex64, device=self.device)

    def new_spectrum(self):
        g = self.grid
        return torch.empty((g.ny, g.nx, self.n_freq), dtype=torch.complex64, device=self.device)

    def reconstruct(self, pos, echo, image=None, echo_scale=1.0, stream=None):
        image = self.new_image() if image is None else image
        sar_reconstruct(self.handle, pos, pos.shape[0], echo, echo_scale, image, self.ws, stream)
        return image

    def spectrum(self, pos, echo, spec=None, echo_scale=1.0, stream=None):
        spec = self.new_spectrum() if spec is None else spec
        sar_spectrum(self.handle, pos, pos.shape[0], echo, echo_scale, spec, self.ws, stream)
        return spec

    def image_from_spectrum(self, spec, image=None, stream=None):
        image = self.new_image() if image is None else image
        sar_image_from_spectrum(self.handle, spec, image, self.ws, stream)
        return image

    def backproject(self, pos, echo, image=None, echo_scale=1.0, stream=None):
        """Direct back-projection on the plan's grid (sar_backproject)."""
        image = self.new_image() if image is None else image
        _check_scan(self.info_struct(), pos, pos.shape[0], echo)
        _check(library().sar_backproject(self.handle, _dptr(pos, "pos", torch.float64), int(pos.shape[0]),
                                         _dptr(echo, "echo"), float(echo_scale),
                                         _dptr(image, "image", torch.complex64, _image_shape(self.info_struct())),
                                         _stream(stream)))
        return image

    def info_struct(self):
        return _info(self.handle)

    def set_grid_tile(self, tile):
        _check(library().sar_plan_set_grid_tile(self.handle, int(tile)))
        self.info = sar_plan_get_info(self.handle)

    def autotune(self, pos, echo, echo_scale=1.0, stream=None):
        """Time the gridding tile configurations on this scan and keep the
        fastest (sar_plan_autotune); returns the chosen configuration."""
        t = ctypes.c_int32()
        _check_scan(self.info_struct(), pos, pos.shape[0], echo)
        _check(library().sar_plan_autotune(self.handle, _dptr(pos, "pos", torch.float64), int(pos.shape[0]),
                                           _dptr(echo, "echo"), float(echo_scale), _dptr(self.ws, "workspace"),
                                           _stream(stream), ctypes.byref(t)))
        self.info = sar_plan_get_info(self.handle)
        return int(t.value)

    def close(self):
        if self.handle is not None:
            sar_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
