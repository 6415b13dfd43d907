"""The compiled piecewise-polynomial form of the Stolt NUFFT's
exponential-of-semicircle kernel (paper_2305_02064_amd/csrc/es_poly.hpp) is the
one its generator writes, and its taps, evaluated in float32, match the kernel
exp(beta (sqrt(1 - z^2) - 1)) to within the kernel's own value at the edge of
its support (or float32 rounding, whichever is larger)."""

import importlib.util
import os
import re

import numpy as np

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2305_02064_amd", "csrc")


def _gen():
    spec = importlib.util.spec_from_file_location("gen_es_poly", os.path.join(CSRC, "gen_es_poly.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_header_is_current():
    with open(os.path.join(CSRC, "es_poly.hpp")) as f:
        assert f.read() == _gen().render()


def test_taps_match_the_kernel():
    with open(os.path.join(CSRC, "es_poly.hpp")) as f:
        txt = f.read()
    for wz, beta, deg in _gen().KERNELS:
        block = txt[txt.index(f"struct EsPoly<{wz}>"):]
        block = block[:block.index("};\n};")]
        rows = re.findall(r"\{([^{}]*)\},", block)
        coef = np.array([[float(v.rstrip("f")) for v in r.split(",")] for r in rows], np.float32)
        assert coef.shape == (wz, deg + 1)
        for tau in np.linspace(0.0, 1.0, 97)[1:]:
            t = np.float32(2 * tau - 1)
            for s in range(wz):
                v = np.float32(0)
                for c in coef[s]:
                    v = np.float32(v * t + c)           # Horner in float32, as the kernel does
                z = 2 * (tau + s - wz / 2) / wz
                ref = np.exp(beta * (np.sqrt(max(1 - z * z, 0.0)) - 1)) if abs(z) <= 1 else 0.0
                # the fit error is about exp(-beta); float32 Horner adds ~1e-7
                assert abs(float(v) - ref) < max(2.5 * np.exp(-beta), 1e-7), (wz, s, tau)
