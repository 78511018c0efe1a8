"""Host-side checks of the C ABI: the library loads, exports every declared
entry point, and its host-only coefficient call is right (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import coeffs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rexi.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\s*\*)\s*(\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    import paper_1812_03431_amd as rexi
    return rexi.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "rexi_step" in names and "sh_forward" in names and len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n


def test_coefficients_match_oracle_as_functions():
    import paper_1812_03431_amd as rexi
    for name in ("t63_single", "t63_jet", "t256_fwd_adj"):
        w = synth.WORKLOADS[name]
        a, bp, bm = rexi.rexi_coeffs(w.M, w.h, w.L)
        assert len(a) == 2 * (w.M + w.L) + 1
        assert np.allclose(a.imag, w.h * np.arange(-(w.M + w.L), w.M + w.L + 1), rtol=0, atol=1e-12)
        co = coeffs.rexi_coefficients(w.M, w.h, w.L)
        xm = 1.001 * np.sqrt(synth.GRAVITY * synth.MEAN_DEPTH * w.T * (w.T + 1)) / synth.EARTH_RADIUS * w.dt
        x = np.linspace(-xm, xm, 3001)
        z = 1j * x[:, None]
        lib_val = (bp / (z + a)).sum(1) + (bm / (a - z)).sum(1)
        assert np.max(np.abs(lib_val - coeffs.rexi_scalar(x, co))) < 2e-12
        # renormalised: x = 0 response exactly one
        assert abs(np.sum((bp + bm) / a) - 1) < 1e-14


def test_coefficient_argument_errors(lib):
    n = ctypes.c_int(0)
    assert lib.rexi_coeffs(0, 0.2, 11, 1, 0, None, None, None, ctypes.byref(n)) == -1
    assert lib.rexi_coeffs(8, -0.2, 11, 1, 0, None, None, None, ctypes.byref(n)) == -1
    assert lib.rexi_coeffs(8, 0.2, 40, 1, 0, None, None, None, ctypes.byref(n)) == -1
    assert lib.rexi_coeffs(8, 0.2, 11, 1, 0, None, None, None, ctypes.byref(n)) == 0
    assert n.value == 39
    buf = (ctypes.c_double * 10)()
    assert lib.rexi_coeffs(8, 0.2, 11, 1, 5, buf, buf, buf, ctypes.byref(n)) == -1
    assert b"capacity" in lib.rexi_last_error()


def test_plan_argument_errors(lib):
    import paper_1812_03431_amd as rexi
    p = rexi.params_for(synth.WORKLOADS["t63_single"])
    h = ctypes.c_void_p()
    bad = rexi.RexiParams.from_buffer_copy(p)
    bad.T = 0
    assert lib.rexi_plan_create(ctypes.byref(bad), ctypes.byref(h)) == -1
    bad = rexi.RexiParams.from_buffer_copy(p)
    bad.nlon = 100
    assert lib.rexi_plan_create(ctypes.byref(bad), ctypes.byref(h)) == -1
    bad = rexi.RexiParams.from_buffer_copy(p)
    bad.dt = -1.0
    assert lib.rexi_plan_create(ctypes.byref(bad), ctypes.byref(h)) == -1
    # the transforms pair latitude rows j and nlat-1-j and hold at most 2048
    # rows: odd or larger nlat is refused by the parameter check, before any
    # device allocation (so it is refused here, without a GPU, as well)
    for nlat in (3, 65, 2050, 4096):
        bad = rexi.RexiParams.from_buffer_copy(p)
        bad.nlat = nlat
        assert lib.rexi_plan_create(ctypes.byref(bad), ctypes.byref(h)) == -1, nlat
        assert b"nlat" in lib.rexi_last_error()
        assert not h.value
    assert lib.rexi_plan_destroy(None) == -1
    assert lib.rexi_step(None, None, None, 1, 1, None) == -1


def test_solve_variant_query():
    # host-only query of the compiled solve variants: the per-term form's are
    # a subset of the batched form's tilings, and every variant tiles with an
    # even number of elements per lane and a known move kind
    import paper_1812_03431_amd as rexi
    v = rexi.solve_variants()
    pt = rexi.solve_variants(per_term=True)
    assert len(v) >= 10 and len(set(v)) == len(v)
    assert {(se, k) for se, k, _ in pt} <= {(se, k) for se, k, _ in v}
    for se, kind, st in v + pt:
        assert se % 2 == 0 and 2 <= se <= 16 and kind in (0, 1, 2) and st >= 1
