"""The input generator's float64 echo synthesis with torch (used on the GPU
for the large scan) against its NumPy form on sampled entries: both write out
the same scattering model (exact ranges, amplitude 1/(R^T R^R)), so they must
agree to rounding.  The large scan's geometry and scene at full size, a subset
of its shots; 10^4 random (shot, pair, frequency) entries."""

import numpy as np
import pytest

from sarsynth import config2_geometry, synth_echo_numpy, synth_echo_torch


def _check(device, n_shots, n_entries):
    import torch
    sc = config2_geometry(0)
    rng = np.random.default_rng(5)
    shots = np.sort(rng.choice(sc.n_pos, n_shots, replace=False))
    pos = sc.pos[shots]
    got = synth_echo_torch(pos, sc.tx_xy, sc.rx_xy, sc.freq, sc.targets, sc.amps, torch.device(device),
                           out_dtype=torch.complex128).cpu().numpy()
    m = rng.integers(0, n_shots, n_entries)
    p = rng.integers(0, got.shape[1], n_entries)
    f = rng.integers(0, got.shape[2], n_entries)
    ref = np.empty(n_entries, np.complex128)
    for i in range(n_entries):
        ref[i] = synth_echo_numpy(pos[m[i]:m[i] + 1], sc.tx_xy, sc.rx_xy, sc.freq[f[i]:f[i] + 1], sc.targets,
                                  sc.amps)[0, p[i], 0]
    err = np.abs(got[m, p, f] - ref).max() / np.abs(ref).max()
    print(f"echo synthesis, {device}: {n_entries} entries, max rel error {err:.2e}")
    assert err <= 1e-12


def test_synth_echo_torch_matches_numpy_cpu():
    _check("cpu", 8, 500)


@pytest.mark.gpu
def test_synth_echo_torch_matches_numpy_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _check("cuda", 64, 10_000)
