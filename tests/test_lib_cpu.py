"""CPU-only checks of the product library: it loads, exports every entry point
the C header declares, and its host-side model compile agrees with the
oracle's compile."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import kan
from paper_2409_07751_amd import compile as pc
from paper_2409_07751_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hekan.h")
LIB = os.path.join(ROOT, "paper_2409_07751_amd", "libhekan.so")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(he_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libhekan.so is not built")
    lib = ctypes.CDLL(LIB)
    names = header_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_header_function():
    from paper_2409_07751_amd import hekan
    declared = set(hekan._SIGS) | {"he_last_error"}
    assert set(header_functions()) == declared


@pytest.mark.parametrize("name", ["tiny", "image"])
def test_product_compile_matches_oracle_compile(name):
    wl = synth.WORKLOADS[name]
    raw = synth.raw_weights(wl)
    calib = synth.calibration_inputs(wl, 256)
    a = pc.compile_kan(raw, calib, wl.silu_degree, [list(c) for c in wl.comp_degrees], wl.grid, wl.silu_range, prescale=wl.prescale)
    b = kan.compile_model(raw, calib, [wl.silu_degree] * len(raw), [list(c) for c in wl.comp_degrees], wl.grid,
                          wl.silu_range, prescale=wl.prescale)
    for La, Lb in zip(a, b):
        assert np.allclose(La.knots, Lb.knots, rtol=1e-12, atol=1e-12)
        assert abs(La.R - Lb.R) < 1e-9 * La.R and La.silu_lo == pytest.approx(Lb.silu_lo) and La.silu_hi == pytest.approx(Lb.silu_hi)
        assert np.abs(La.silu_coeffs - Lb.silu_coeffs).max() < 1e-7
        for sa, sb in zip(La.comp, Lb.comp):
            assert np.allclose(sa, sb, rtol=1e-12, atol=0)
    x = synth.inputs(wl, 3)
    assert np.abs(pc.plain_forward(x, a) - kan.he_friendly_kan(x, b)).max() < 1e-6
