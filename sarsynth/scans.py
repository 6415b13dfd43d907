"""Seeded synthetic scans shaped like the paper's workloads.

Every scan is reproducible from (config id, seed).  The echo model is the
frequency-domain Born model of Sec. II-C with an isotropic antenna and
P(f) = 1:

    s(n, f) = sum_t  a_t / (R_T R_R) * exp(-j k (R_T + R_R)),   k = 2 pi f / c,

where R_T and R_R are the exact Tx and Rx ranges of Sec. II-B.  Noise is
circular complex Gaussian at a stated SNR = mean |s|^2 / sigma^2.

Layouts used by both the oracle and the GPU library:
    pos   [N_pos, 3]  float64   device origin of each shot (m)
    tx_xy [n_tx, 2]   float64   Tx offsets from the origin, z offset 0
    rx_xy [n_rx, 2]   float64   Rx offsets from the origin, z offset 0
    freq  [N_f]       float64   strictly increasing (Hz)
    echo  [N_pos, n_tx*n_rx, N_f] complex64, pair index = t*n_rx + r
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

C0 = 299_792_458.0  # speed of light in vacuum (m/s)
FC = 79e9           # centre of the 77-81 GHz sweep of the prototype (Sec. IV)
LAMBDA_C = C0 / FC  # about 3.79 mm (Sec. V-A)


@dataclass
class ImageGrid:
    """Voxel (u, v, w) sits at (x0 + u*dx, y0 + v*dy, z0 + w*dz).

    z_ref is the projection plane Z_0 of Sec. II-B; z_focus is the scene
    reference depth used for the multistatic term of the residual path.
    """

    nx: int
    ny: int
    nz: int
    x0: float
    y0: float
    z0: float
    dx: float
    dy: float
    dz: float
    z_ref: float = 0.0
    z_focus: float = 0.3

    @property
    def n_voxels(self) -> int:
        return self.nx * self.ny * self.nz

    def coords(self):
        return (self.x0 + self.dx * np.arange(self.nx),
                self.y0 + self.dy * np.arange(self.ny),
                self.z0 + self.dz * np.arange(self.nz))


@dataclass
class Scan:
    pos: np.ndarray
    tx_xy: np.ndarray
    rx_xy: np.ndarray
    freq: np.ndarray
    grid: ImageGrid
    echo: Optional[object] = None            # numpy complex64 or torch tensor
    targets: Optional[np.ndarray] = None     # [T, 3]
    amps: Optional[np.ndarray] = None        # [T] complex128
    meta: dict = field(default_factory=dict)

    @property
    def n_pos(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_pair(self) -> int:
        return int(self.tx_xy.shape[0] * self.rx_xy.shape[0])

    @property
    def n_freq(self) -> int:
        return int(self.freq.shape[0])


def awr1443_layout(fc: float = FC):
    """2 Tx spaced 2*lambda_c and 4 Rx spaced lambda_c/2 (Sec. IV), laid out
    collinear along y and centred on the device origin: Tx y = +-lambda_c,
    Rx y = {-3,-1,1,3} lambda_c/4, all x = 0."""
    lam = C0 / fc
    tx = np.array([[0.0, -lam], [0.0, lam]])
    rx = np.array([[0.0, -0.75 * lam], [0.0, -0.25 * lam],
                   [0.0, 0.25 * lam], [0.0, 0.75 * lam]])
    return tx, rx


def sweep(n_freq: int, f_start: float = 77e9, f_stop: float = 81e9):
    """Stepped-frequency sweep over the prototype's band, end points included."""
    return np.linspace(f_start, f_stop, n_freq, dtype=np.float64)


def _rng(config_id: int, seed: int):
    return np.random.default_rng(np.random.SeedSequence([int(config_id), int(seed)]))


# ----------------------------------------------------------------------------
# echo synthesis (forward model only)
# ----------------------------------------------------------------------------

def synth_echo_numpy(pos, tx_xy, rx_xy, freq, tgt, amp, chunk=256):
    """Echo cube [N_pos, n_tx*n_rx, N_f] (complex128) of point scatterers."""
    pos = np.asarray(pos, np.float64)
    k = 2.0 * np.pi * np.asarray(freq, np.float64) / C0
    n_pos, n_tx, n_rx, nf = pos.shape[0], tx_xy.shape[0], rx_xy.shape[0], k.shape[0]
    out = np.zeros((n_pos, n_tx * n_rx, nf), np.complex128)
    tgt = np.asarray(tgt, np.float64)
    amp = np.asarray(amp, np.complex128)
    for m0 in range(0, n_pos, chunk):
        p = pos[m0:m0 + chunk]
        dz2 = (p[:, None, 2] - tgt[None, :, 2]) ** 2                       # [m, T]
        tx = p[:, None, :2] + tx_xy[None, :, :]                            # [m, nt, 2]
        rx = p[:, None, :2] + rx_xy[None, :, :]
        rt = np.sqrt((tx[:, :, None, 0] - tgt[None, None, :, 0]) ** 2 +
                     (tx[:, :, None, 1] - tgt[None, None, :, 1]) ** 2 + dz2[:, None, :])
        rr = np.sqrt((rx[:, :, None, 0] - tgt[None, None, :, 0]) ** 2 +
                     (rx[:, :, None, 1] - tgt[None, None, :, 1]) ** 2 + dz2[:, None, :])
        r = rt[:, :, None, :] + rr[:, None, :, :]                          # [m, nt, nr, T]
        a = amp[None, None, None, :] / (rt[:, :, None, :] * rr[:, None, :, :])
        ph = np.exp(-1j * r[..., None] * k)                               # [m, nt, nr, T, f]
        out[m0:m0 + chunk] = np.einsum('abct,abctf->abcf', a, ph).reshape(p.shape[0], n_tx * n_rx, nf)
    return out


def synth_echo_torch(pos, tx_xy, rx_xy, freq, tgt, amp, device, pos_chunk=256, tgt_chunk=128,
                     out_dtype=None):
    """Same model as synth_echo_numpy, evaluated in float64 with torch on
    `device` (used for the large scans whose direct synthesis is too slow on
    a CPU).  Returns a complex64 tensor on `device`."""
    import torch
    f64 = torch.float64
    posd = torch.as_tensor(np.asarray(pos), dtype=f64, device=device)
    txd = torch.as_tensor(np.asarray(tx_xy), dtype=f64, device=device)
    rxd = torch.as_tensor(np.asarray(rx_xy), dtype=f64, device=device)
    k = torch.as_tensor(2.0 * np.pi * np.asarray(freq, np.float64) / C0, dtype=f64, device=device)
    tg = torch.as_tensor(np.asarray(tgt), dtype=f64, device=device)
    am = torch.as_tensor(np.asarray(amp), dtype=torch.complex128, device=device)
    n_pos, n_tx, n_rx, nf = posd.shape[0], txd.shape[0], rxd.shape[0], k.shape[0]
    out = torch.empty((n_pos, n_tx * n_rx, nf), dtype=out_dtype or torch.complex64, device=device)
    for m0 in range(0, n_pos, pos_chunk):
        p = posd[m0:m0 + pos_chunk]
        m = p.shape[0]
        acc = torch.zeros((m, n_tx, n_rx, nf), dtype=torch.complex128, device=device)
        tx = p[:, None, :2] + txd[None]
        rx = p[:, None, :2] + rxd[None]
        for t0 in range(0, tg.shape[0], tgt_chunk):
            t = tg[t0:t0 + tgt_chunk]
            a = am[t0:t0 + tgt_chunk]
            dz2 = (p[:, None, 2] - t[None, :, 2]) ** 2
            rt = torch.sqrt((tx[:, :, None, 0] - t[None, None, :, 0]) ** 2 +
                            (tx[:, :, None, 1] - t[None, None, :, 1]) ** 2 + dz2[:, None, :])
            rr = torch.sqrt((rx[:, :, None, 0] - t[None, None, :, 0]) ** 2 +
                            (rx[:, :, None, 1] - t[None, None, :, 1]) ** 2 + dz2[:, None, :])
            r = rt[:, :, None, :] + rr[:, None, :, :]                      # [m, nt, nr, T]
            w = a[None, None, None, :] / (rt[:, :, None, :] * rr[:, None, :, :])
            ph = torch.polar(torch.ones((), dtype=f64, device=device), -r[..., None] * k)  # [m,nt,nr,T,f]
            acc += (w[..., None] * ph).sum(dim=3)
        out[m0:m0 + m] = acc.reshape(m, n_tx * n_rx, nf).to(out.dtype)
    return out


def add_noise_numpy(echo, snr_db, rng):
    """Circular complex Gaussian noise; SNR = mean|s|^2 / sigma^2 over the cube."""
    p = float(np.mean(np.abs(echo) ** 2))
    sigma = np.sqrt(p / (10.0 ** (snr_db / 10.0)))
    n = rng.standard_normal(echo.shape) + 1j * rng.standard_normal(echo.shape)
    return echo + (sigma / np.sqrt(2.0)) * n


def add_noise_torch(echo, snr_db, seed):
    import torch
    p = float((echo.real.float() ** 2 + echo.imag.float() ** 2).mean().item())
    sigma = (p / (10.0 ** (snr_db / 10.0))) ** 0.5
    g = torch.Generator(device=echo.device)
    g.manual_seed(int(seed))
    nr = torch.randn(echo.shape, generator=g, device=echo.device, dtype=torch.float32)
    ni = torch.randn(echo.shape, generator=g, device=echo.device, dtype=torch.float32)
    echo += torch.complex(nr, ni).to(echo.dtype) * (sigma / 2.0 ** 0.5)
    return echo


# ----------------------------------------------------------------------------
# trajectories and scenes
# ----------------------------------------------------------------------------

def _smooth_walk(rng, n, taps, sigma):
    """Gaussian random walk, moving-average low-passed, rescaled to std sigma."""
    w = np.cumsum(rng.standard_normal(n + taps))
    w = np.convolve(w, np.ones(taps) / taps, mode='valid')[:n]
    w = w - w.mean()
    s = w.std()
    return w * (sigma / s) if s > 0 else w


def _smooth_noise2d(rng, n0, n1, width):
    a = rng.standard_normal((n0 + 2 * width, n1 + 2 * width))
    ker = np.ones(width) / width
    a = np.apply_along_axis(lambda r: np.convolve(r, ker, mode='same'), 0, a)
    a = np.apply_along_axis(lambda r: np.convolve(r, ker, mode='same'), 1, a)
    return a[width:width + n0, width:width + n1]


def config1_scan(seed: int = 0, snr_db: float = 20.0, with_echo: bool = True) -> Scan:
    """Tiny plain scan: 2Tx x 4Rx, 32 frequencies over 77-81 GHz, 32 x 16
    jittered planar positions (x step lambda/4, y step 8 lambda, x/y jitter
    U(+-lambda/8), z ~ U(+-3 mm)), 3 point scatterers at z in [0.25, 0.35] m;
    image 32 x 32 x 16 voxels over x, y in [-0.1, 0.1) and z in [0.2, 0.4)."""
    rng = _rng(1, seed)
    lam = LAMBDA_C
    tx, rx = awr1443_layout()
    freq = sweep(32)
    ix, iy = np.meshgrid(np.arange(32), np.arange(16), indexing='ij')
    x = (ix.ravel() - 15.5) * lam / 4 + rng.uniform(-lam / 8, lam / 8, ix.size)
    y = (iy.ravel() - 7.5) * 8 * lam + rng.uniform(-lam / 8, lam / 8, ix.size)
    z = rng.uniform(-3e-3, 3e-3, ix.size)
    pos = np.stack([x, y, z], axis=1)
    grid = ImageGrid(nx=32, ny=32, nz=16, x0=-0.1, y0=-0.1, z0=0.2,
                     dx=0.2 / 32, dy=0.2 / 32, dz=0.2 / 16, z_ref=0.0, z_focus=0.3)
    tgt = np.stack([rng.uniform(-0.06, 0.06, 3), rng.uniform(-0.06, 0.06, 3),
                    rng.uniform(0.25, 0.35, 3)], axis=1)
    amp = np.exp(1j * rng.uniform(0, 2 * np.pi, 3))
    scan = Scan(pos=pos, tx_xy=tx, rx_xy=rx, freq=freq, grid=grid, targets=tgt, amps=amp,
                meta={"config": "tiny-32x16", "seed": seed, "snr_db": snr_db})
    if with_echo:
        e = synth_echo_numpy(pos, tx, rx, freq, tgt, amp)
        scan.echo = add_noise_numpy(e, snr_db, rng).astype(np.complex64)
    return scan


def clustered_scan(seed: int = 0, n_dwell: int = 4608, snr_db: float = 20.0, n_freq: int = 32) -> Scan:
    """The tiny scan's 512 shots plus n_dwell shots at one position (a hand
    that pauses in the middle of the aperture, the extreme of irregular
    freehand sampling): every pair of those shots lands on the same virtual
    element, so eight cells of the gridding grid hold n_dwell samples each.
    Scene and image as the tiny scan; n_freq frequencies over 77-81 GHz."""
    base = config1_scan(seed, snr_db, with_echo=False)
    if n_freq != len(base.freq):
        base.freq = sweep(n_freq)
    rng = _rng(6, seed)
    dwell = np.tile(base.pos[len(base.pos) // 2], (n_dwell, 1))
    pos = np.concatenate([base.pos, dwell], axis=0)
    scan = Scan(pos=pos, tx_xy=base.tx_xy, rx_xy=base.rx_xy, freq=base.freq, grid=base.grid,
                targets=base.targets, amps=base.amps,
                meta={"config": f"clustered-tiny+{n_dwell}", "seed": seed, "snr_db": snr_db})
    e = synth_echo_numpy(pos, base.tx_xy, base.rx_xy, base.freq, base.targets, base.amps)
    scan.echo = add_noise_numpy(e, snr_db, rng).astype(np.complex64)
    return scan


def config2_geometry(seed: int = 0, n_rows: int = 256, n_cols: int = 512, n_freq: int = 256,
                     nz: int = 256) -> Scan:
    """Large freehand scan geometry and scene (no echo): n_rows serpentine rows
    (y) x n_cols shots (x) at nominal pitch lambda/4, x/y deviation a smoothed
    random walk with std lambda/4, z deviation the same with std 1 cm clipped
    to +-2 cm; 200 random points in the central 80% of the image volume plus an
    extended surface (2 mm lattice, smooth +-5 mm height field at 0.3 m, kept
    where a smoothed random mask exceeds its 70th percentile); image
    n_cols x n_rows x nz at lambda/4 laterally and 1 mm in z from 0.172 m."""
    rng = _rng(2, seed)
    lam = LAMBDA_C
    pitch = lam / 4
    tx, rx = awr1443_layout()
    freq = sweep(n_freq)
    n = n_rows * n_cols
    row = np.repeat(np.arange(n_rows), n_cols)
    col = np.tile(np.arange(n_cols), n_rows)
    col = np.where(row % 2 == 0, col, n_cols - 1 - col)        # serpentine order
    x = (col - (n_cols - 1) / 2) * pitch + _smooth_walk(rng, n, 64, lam / 4)
    y = (row - (n_rows - 1) / 2) * pitch + _smooth_walk(rng, n, 64, lam / 4)
    z = np.clip(_smooth_walk(rng, n, 64, 0.01), -0.02, 0.02)
    pos = np.stack([x, y, z], axis=1)
    dz = 1e-3
    grid = ImageGrid(nx=n_cols, ny=n_rows, nz=nz, x0=-(n_cols // 2) * pitch, y0=-(n_rows // 2) * pitch,
                     z0=0.172, dx=pitch, dy=pitch, dz=dz, z_ref=0.0, z_focus=0.3)
    ext = np.array([n_cols * pitch, n_rows * pitch, nz * dz])
    lo = np.array([grid.x0, grid.y0, grid.z0]) + 0.1 * ext
    pts = lo + 0.8 * ext * rng.uniform(0, 1, (200, 3))
    # extended surface on a 12 x 12 cm patch
    ns = 60
    mask = _smooth_noise2d(rng, ns, ns, 6)
    keep = mask > np.quantile(mask, 0.7)
    h = _smooth_noise2d(rng, ns, ns, 10)
    h = 5e-3 * h / np.max(np.abs(h))
    sx, sy = np.meshgrid((np.arange(ns) - ns / 2) * 2e-3, (np.arange(ns) - ns / 2) * 2e-3, indexing='ij')
    surf = np.stack([sx[keep], sy[keep], 0.3 + h[keep]], axis=1)
    tgt = np.concatenate([pts, surf], axis=0)
    amp = (rng.standard_normal(tgt.shape[0]) + 1j * rng.standard_normal(tgt.shape[0])) / np.sqrt(2)
    return Scan(pos=pos, tx_xy=tx, rx_xy=rx, freq=freq, grid=grid, targets=tgt, amps=amp,
                meta={"config": f"freehand-{n_cols}x{n_rows}", "seed": seed})


def config2_scan(seed: int = 0, device=None, snr_db: float = 20.0, **kw) -> Scan:
    """config2_geometry plus its echo synthesised in float64 on `device`
    (a torch device) and stored complex64 there."""
    scan = config2_geometry(seed, **kw)
    e = synth_echo_torch(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.targets, scan.amps, device)
    scan.echo = add_noise_torch(e, snr_db, seed=1_000_003 * (seed + 1))
    scan.meta["snr_db"] = snr_db
    return scan


def _snap_235(s: int, lo: int = 64, hi: int = 256) -> int:
    """Nearest 2^a 3^b 5^c in [lo, hi] (ties to the smaller)."""
    cands = sorted({2 ** a * 3 ** b * 5 ** c for a in range(0, 9) for b in range(0, 6) for c in range(0, 4)
                    if lo <= 2 ** a * 3 ** b * 5 ** c <= hi})
    return min(cands, key=lambda v: (abs(v - s), v))


def config4_scan(seed: int, with_echo: bool = True, device=None) -> Scan:
    """One scan of the uneven batch: side s log-uniform in [64, 256] snapped to
    a 2^a 3^b 5^c size, s x s positions at lambda/4, N_f in {64, 128, 256},
    smooth z deviation scaled to max |d_z| = A ~ U(1, 2) cm, 20-100 points at
    z in [0.2, 0.5] m.  The image is sized to the aperture: s x s x N_f voxels
    at lambda/4 laterally, centred on it, z in [0.2, 0.5)."""
    rng = _rng(4, seed)
    lam = LAMBDA_C
    pitch = lam / 4
    s = _snap_235(int(round(2 ** rng.uniform(6, 8))))
    nf = int(rng.choice([64, 128, 256]))
    tx, rx = awr1443_layout()
    freq = sweep(nf)
    n = s * s
    row = np.repeat(np.arange(s), s)
    col = np.tile(np.arange(s), s)
    col = np.where(row % 2 == 0, col, s - 1 - col)
    x = (col - (s - 1) / 2) * pitch + _smooth_walk(rng, n, 32, lam / 8)
    y = (row - (s - 1) / 2) * pitch + _smooth_walk(rng, n, 32, lam / 8)
    a = rng.uniform(0.01, 0.02)
    zw = _smooth_walk(rng, n, 32, 1.0)
    z = zw * (a / np.max(np.abs(zw)))
    pos = np.stack([x, y, z], axis=1)
    nt = int(rng.integers(20, 101))
    ext = s * pitch
    tgt = np.stack([rng.uniform(-0.4 * ext, 0.4 * ext, nt), rng.uniform(-0.4 * ext, 0.4 * ext, nt),
                    rng.uniform(0.2, 0.5, nt)], axis=1)
    amp = (rng.standard_normal(nt) + 1j * rng.standard_normal(nt)) / np.sqrt(2)
    side = s
    grid = ImageGrid(nx=side, ny=side, nz=nf, x0=-(side // 2) * pitch, y0=-(side // 2) * pitch, z0=0.2,
                     dx=pitch, dy=pitch, dz=0.3 / nf, z_ref=0.0, z_focus=0.35)
    scan = Scan(pos=pos, tx_xy=tx, rx_xy=rx, freq=freq, grid=grid, targets=tgt, amps=amp,
                meta={"config": f"batched-{s}x{s}x{nf}", "seed": seed})
    if with_echo:
        if device is None:
            e = synth_echo_numpy(pos, tx, rx, freq, tgt, amp)
            scan.echo = add_noise_numpy(e, 20.0, rng).astype(np.complex64)
        else:
            e = synth_echo_torch(pos, tx, rx, freq, tgt, amp, device)
            scan.echo = add_noise_torch(e, 20.0, seed=7_000_003 * (seed + 1))
    return scan


def point_scan(nx_pos: int, ny_pos: int, pitch: float, target, n_freq: int, grid: ImageGrid,
               tx_xy=None, rx_xy=None, z_dev=None, seed: int = 0, jitter: float = 0.0,
               f_start: float = 77e9, f_stop: float = 81e9, z_track: str = "uniform") -> Scan:
    """Planar (optionally jittered / multi-planar) lattice of shots around the
    origin imaging one unit point scatterer; monostatic unless a layout is
    given.  z_dev: None, or the largest z deviation max |d^z| (m), drawn per
    z_track: "uniform" (independent per shot, uniform in +-z_dev) or "curve"
    (a semi-smooth random curve over the shots in order: a low-passed random
    walk plus 10% white roughness, zero mean, scaled so that max |d^z| = z_dev,
    the freehand tracks of Sec. V-A)."""
    rng = _rng(9, seed)
    if tx_xy is None:
        tx_xy = np.zeros((1, 2))
    if rx_xy is None:
        rx_xy = np.zeros((1, 2))
    ix, iy = np.meshgrid(np.arange(nx_pos), np.arange(ny_pos), indexing='ij')
    x = (ix.ravel() - (nx_pos - 1) / 2) * pitch
    y = (iy.ravel() - (ny_pos - 1) / 2) * pitch
    if jitter:
        x = x + rng.uniform(-jitter, jitter, x.size)
        y = y + rng.uniform(-jitter, jitter, y.size)
    if not z_dev:
        z = np.zeros_like(x)
    elif z_track == "uniform":
        z = rng.uniform(-z_dev, z_dev, x.size)
    elif z_track == "curve":
        z = _smooth_walk(rng, x.size, 24, 1.0)
        z = z + 0.1 * rng.standard_normal(x.size)
        z = z - z.mean()
        z = z * (z_dev / np.max(np.abs(z)))
    else:
        raise ValueError(f"unknown z_track {z_track!r}")
    pos = np.stack([x, y, z], axis=1)
    freq = sweep(n_freq, f_start, f_stop)
    tgt = np.asarray(target, np.float64).reshape(1, 3)
    amp = np.ones(1, np.complex128)
    echo = synth_echo_numpy(pos, tx_xy, rx_xy, freq, tgt, amp)
    return Scan(pos=pos, tx_xy=np.asarray(tx_xy, float), rx_xy=np.asarray(rx_xy, float), freq=freq,
                grid=grid, echo=echo, targets=tgt, amps=amp, meta={"config": "point"})


def depth_pair_scan(n_side: int = 32, n_freq: int = 16, depths=(0.15, 0.45)) -> Scan:
    """Two unit point scatterers on the array axis at the given depths, seen by
    a wide-baseline array (Tx at x = -3, +3 cm, Rx at x = -1, +1 cm: Tx/Rx
    separations of 2 and 4 cm) from a flat n_side x n_side lattice of shots at
    lambda_c/4.  Image 32 x 32 x 16 voxels, lambda_c/4 laterally around the
    axis, z in [0.1, 0.5) at 25 mm, reference depth 0.3 m (the volume's
    centre): a scene whose near target keeps a large multistatic residual
    under a single reference depth."""
    lam = C0 / 79e9
    pitch = lam / 4
    tx = np.array([[-0.03, 0.0], [0.03, 0.0]])
    rx = np.array([[-0.01, 0.0], [0.01, 0.0]])
    a = (np.arange(n_side) - (n_side - 1) / 2) * pitch
    xx, yy = np.meshgrid(a, a, indexing='ij')
    pos = np.stack([xx.ravel(), yy.ravel(), np.zeros(xx.size)], axis=1)
    freq = sweep(n_freq)
    tgt = np.array([[0.0, 0.0, z] for z in depths])
    amp = np.ones(len(depths), np.complex128)
    echo = synth_echo_numpy(pos, tx, rx, freq, tgt, amp)
    grid = ImageGrid(nx=32, ny=32, nz=16, x0=-16 * pitch, y0=-16 * pitch, z0=0.1, dx=pitch, dy=pitch, dz=0.025,
                     z_ref=0.0, z_focus=0.3)
    return Scan(pos=pos, tx_xy=tx, rx_xy=rx, freq=freq, grid=grid, echo=echo, targets=tgt, amps=amp,
                meta={"config": "depth-pair"})
