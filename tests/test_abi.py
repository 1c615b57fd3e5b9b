"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, and its host-only paths (validation, sizes, finite-difference
weights) behave as documented. No kernel is launched."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2406_08923_amd as S
from closed_forms import central_weights

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(stencil_\w+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("stencil_plan", "stencil_apply", "stencil_plan_destroy", "stencil_last_error",
                 "stencil_halo_periodic", "stencil_padded_elems"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = S.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_version_and_padded_elems():
    L = S.lib()
    assert L.stencil_version() >= 10000
    assert S.padded_elems((512, 512, 512), 3) == 518 ** 3
    assert S.padded_elems((2 ** 20,), 1) == 2 ** 20 + 2
    assert S.padded_elems((7, 5), 2) == 11 * 9
    dims = (ctypes.c_int * 3)(4, 4, 4)
    assert L.stencil_padded_elems(4, dims, 1) == 0
    assert L.stencil_padded_elems(3, dims, -1) == 0


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_fd_weights_match_exact_rationals(order, r):
    w = S.fd_weights(order, r)
    exact = np.array([float(v) for v in central_weights(order, r)])
    assert np.max(np.abs(w - exact)) <= 4e-16 * np.max(np.abs(exact))
    if order == 1:
        assert w[r] == 0.0 and np.array_equal(w, -w[::-1])
    else:
        assert np.array_equal(w, w[::-1])


def _plan_rc(**kw):
    d = S._Desc()
    d.ndim = kw.get("ndim", 3)
    dims = kw.get("dims", (8, 8, 8))
    d.dims = (ctypes.c_int * 3)(*dims)
    d.radius = kw.get("radius", 1)
    coeffs = kw.get("coeffs", np.ones(27))
    d.coeffs = None if coeffs is None else coeffs.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.dtype = kw.get("dtype", S.F64)
    d.bc = kw.get("bc", S.PERIODIC)
    d.variant = kw.get("variant", S.VARIANT_AUTO)
    d.row_pitch = kw.get("row_pitch", 0)
    d.x_offset = kw.get("x_offset", 0)
    d.op = kw.get("op", 0)
    h = ctypes.c_void_p()
    return S.lib().stencil_plan(ctypes.byref(d), ctypes.byref(h))


@pytest.mark.parametrize("kw", [dict(ndim=4), dict(ndim=0), dict(radius=9), dict(radius=-1),
                                dict(coeffs=None), dict(dtype=7), dict(bc=3),
                                dict(dims=(2, 8, 8), radius=3, coeffs=np.ones(343)),
                                dict(dims=(0, 8, 8)), dict(variant=9),
                                dict(ndim=1, dims=(4096, 1, 1), radius=1025, coeffs=np.ones(2051)),
                                dict(ndim=2, dims=(64, 64, 1), radius=9, coeffs=np.ones(361)),
                                dict(op=4), dict(op=-1),
                                # layout: x_offset below the radius, pitch too short
                                # for x_offset + nx + r, pitch on a 1-D field, negatives
                                dict(radius=2, x_offset=1, coeffs=np.ones(125)),
                                dict(row_pitch=12, x_offset=4),
                                dict(ndim=1, row_pitch=16, coeffs=np.ones(3)),
                                dict(row_pitch=-1), dict(x_offset=-2)])
def test_plan_rejects_bad_descriptors_without_a_device(kw):
    assert _plan_rc(**kw) == -1
    assert S.lib().stencil_last_error()


def test_plan_rejects_nonfinite_coefficients_before_the_device():
    c = np.ones(27)
    c[3] = np.nan
    assert _plan_rc(coeffs=c) == -1
    c[3] = np.inf
    assert _plan_rc(coeffs=c) == -1


def test_copy_and_halo_validate_before_launch():
    L = S.lib()
    assert L.stencil_copy(ctypes.c_void_p(4096), ctypes.c_void_p(8192), 24, None) == -1
    assert L.stencil_copy(ctypes.c_void_p(4096), ctypes.c_void_p(4096 + 16), 64, None) == -1
    assert L.stencil_copy(ctypes.c_void_p(4104), ctypes.c_void_p(1 << 20), 64, None) == -1
    dims = (ctypes.c_int * 3)(8, 8, 8)
    assert L.stencil_halo_periodic(3, dims, 1, 9, ctypes.c_void_p(4096), None) == -1
    assert L.stencil_halo_periodic(3, dims, 1, 0, None, None) == -1
    assert L.stencil_halo_periodic(3, dims, 9, 0, ctypes.c_void_p(4096), None) == -1


def test_apply_rejects_null_plan():
    assert S.lib().stencil_apply(None, ctypes.c_void_p(4096), ctypes.c_void_p(8192), 1,
                                 None) == -1


def test_layout_helper_aligns_rows():
    from paper_2406_08923_amd.workloads import aligned_layout
    assert aligned_layout(512, 3, 8) == (544, 16)
    assert aligned_layout(512, 3, 4) == (576, 32)
    assert aligned_layout(100, 40, 8) == (192, 48)
    for nx, r, es in [(7, 3, 2), (512, 8, 8), (1, 1, 4)]:
        pitch, ox = aligned_layout(nx, r, es)
        assert ox >= r and pitch >= ox + nx + r
        assert (ox * es) % 128 == 0 and (pitch * es) % 128 == 0
    assert S.lib().stencil_plan_padded_elems(None) == 0


def _rk_rc(**kw):
    d = S._RkDesc()
    d.model = kw.get("model", S.MODEL_MHD8)
    d.ndim = kw.get("ndim", 3)
    d.dims = (ctypes.c_int * 3)(*kw.get("dims", (16, 16, 16)))
    d.precision = kw.get("precision", S.PREC_F64)
    d.ds = (ctypes.c_double * 3)(0.1, 0.1, 0.1)
    d.nu, d.eta, d.cs2 = 1e-3, 1e-3, 1.0
    d.block = (ctypes.c_int * 3)(*kw.get("block", (0, 0, 0)))
    d.variant = kw.get("variant", 0)
    for k, v in dict(S.MHD_FULL_DEFAULTS, **kw.get("mhd", {})).items():
        setattr(d, k, v)
    if "cs2" in kw:
        d.cs2 = kw["cs2"]
    d.mixed = kw.get("mixed", 0)
    h = ctypes.c_void_p()
    return S.lib().stencil_plan_rk(ctypes.byref(d), ctypes.byref(h))


@pytest.mark.parametrize("kw,code", [
    (dict(variant=3), -1),                                  # unknown bank
    (dict(variant=-1), -1),
    (dict(model=S.MODEL_ADVDIFF, ndim=2, dims=(16, 16, 1), variant=S.RK_LDS), -3),  # 3-D only
    (dict(model=S.MODEL_ADVDIFF, variant=S.RK_LDS, block=(64, 16, 32)), -1),  # z planes only
    (dict(variant=S.RK_LDS, block=(16, 8, 2)), -1),         # brick not built
    (dict(variant=S.RK_LDS, block=(64, 4, 1)), -1),
    (dict(variant=S.RK_CACHED, block=(64, 4, 2)), -1),      # one plane per workgroup
    (dict(variant=S.RK_CACHED, block=(48, 1, 0)), -1),      # not a multiple of 64 lanes
    (dict(ndim=2, dims=(16, 16, 1)), -1),                   # MHD8 is 3-D
    (dict(model=3), -1),                                    # unknown model
    (dict(model=S.MODEL_MHD_FULL, ndim=2, dims=(16, 16, 1)), -1),  # 3-D
    (dict(model=S.MODEL_MHD_FULL, mhd=dict(mu0=0.0)), -1),  # closure constants
    (dict(model=S.MODEL_MHD_FULL, mhd=dict(gamma=1.0)), -1),
    (dict(model=S.MODEL_MHD_FULL, mhd=dict(cp=-1.0)), -1),
    (dict(model=S.MODEL_MHD_FULL, cs2=0.0), -1),
    (dict(model=S.MODEL_MHD_FULL, mhd=dict(K=float("nan"))), -1),
    (dict(model=S.MODEL_MHD_FULL, mhd=dict(heat=float("inf"))), -1),
    (dict(model=S.MODEL_MHD_FULL, variant=S.RK_LDS, block=(16, 8, 2)), -1),
    (dict(mixed=2), -1),                                    # unknown mixed form
    (dict(mixed=-1), -1),
    (dict(model=S.MODEL_ADVDIFF, mixed=S.MIXED_DIAGONAL), -1),  # no mixed terms
])
def test_rk_plan_rejects_bad_descriptors_without_a_device(kw, code):
    assert _rk_rc(**kw) == code
    assert S.lib().stencil_last_error()


@pytest.mark.parametrize("kw", [dict(x_offset=2), dict(x_offset=8, row_pitch=20),
                                dict(row_pitch=-4), dict(x_offset=-1)])
def test_rk_plan_rejects_bad_layouts_without_a_device(kw):
    d = S._RkDesc()
    d.model, d.ndim = S.MODEL_MHD8, 3
    d.dims = (ctypes.c_int * 3)(16, 16, 16)
    d.precision = S.PREC_F64
    d.ds = (ctypes.c_double * 3)(0.1, 0.1, 0.1)
    d.nu, d.eta, d.cs2 = 1e-3, 1e-3, 1.0
    d.row_pitch = kw.get("row_pitch", 0)
    d.x_offset = kw.get("x_offset", 0)
    h = ctypes.c_void_p()
    assert S.lib().stencil_plan_rk(ctypes.byref(d), ctypes.byref(h)) == -1


def test_full_mhd_constants_are_ignored_by_the_proxy_model():
    # the proxy plan reaches device selection (no GPU here) instead of
    # rejecting closure constants it does not read
    rc = _rk_rc(model=S.MODEL_MHD8, mhd=dict(mu0=0.0, gamma=0.5))
    assert rc != -1


def test_rk_plan_rejects_unknown_mhd_constant_names():
    with pytest.raises(ValueError):
        S.RkPlan(S.MODEL_MHD_FULL, (8, 8, 8), mhd=dict(kappa=1.0))


def test_energy_rejects_a_missing_plan_without_a_device():
    out = (ctypes.c_double * 2)()
    assert S.lib().stencil_energy(None, None, S.F64, out, None) == -1
    assert S.lib().stencil_last_error()
