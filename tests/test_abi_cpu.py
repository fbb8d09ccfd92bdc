"""The C ABI library on the CPU: it loads, exports every declared symbol and rejects bad arguments
before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "green_gw.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(green_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2406_18479_amd import _lib
    return _lib


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for n in ["green_gw_polarization", "green_gw_screen", "green_gw_selfenergy", "green_dyson", "green_gw_iterate",
              "green_plan_create", "green_plan_destroy", "green_workspace_bytes", "green_strerror"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib.LIB, name), name
        assert isinstance(getattr(lib.LIB, name), ctypes._CFuncPtr)


def test_strerror(lib):
    assert lib.LIB.green_strerror(0) == b"success"
    assert b"workspace" in lib.LIB.green_strerror(-2)
    assert lib.LIB.green_strerror(12345) == b"unknown status"


def _dims(lib, **kw):
    d = dict(kmesh=(1, 1, 1), nao=4, naux=8, ntau=8, nw_f=8, nw_b=9, nspin=1, beta=10.0)
    d.update(kw)
    return lib.Dims((ctypes.c_int32 * 3)(*d["kmesh"]), d["nao"], d["naux"], d["ntau"], d["nw_f"], d["nw_b"],
                    d["nspin"], d["beta"])


def _grid(lib, ntau=8):
    arrs = [np.zeros(ntau), np.zeros(ntau), np.zeros(ntau + 1)] + [np.zeros((ntau + 1, ntau), complex)] * 4
    return lib.GridC(*[a.ctypes.data for a in arrs]), arrs


@pytest.mark.parametrize("bad", [dict(nao=0), dict(nao=600), dict(naux=513), dict(ntau=7, nw_f=7, nw_b=8),
                                 dict(nw_f=9), dict(nw_b=8), dict(nspin=3), dict(beta=-1.0), dict(kmesh=(0, 1, 1))])
def test_plan_create_rejects_bad_dims(lib, bad):
    g, keep = _grid(lib)
    h = ctypes.c_void_p()
    st = lib.LIB.green_plan_create(ctypes.byref(_dims(lib, **bad)), ctypes.byref(g), 0, 0, ctypes.byref(h))
    assert st == -1 and not h.value
    del keep


def test_plan_create_rejects_null_and_unknown_precision(lib):
    g, keep = _grid(lib)
    h = ctypes.c_void_p()
    assert lib.LIB.green_plan_create(None, ctypes.byref(g), 0, 0, ctypes.byref(h)) == -1
    assert lib.LIB.green_plan_create(ctypes.byref(_dims(lib)), None, 0, 0, ctypes.byref(h)) == -1
    assert lib.LIB.green_plan_create(ctypes.byref(_dims(lib)), ctypes.byref(g), 0, 0, None) == -1
    assert lib.LIB.green_plan_create(ctypes.byref(_dims(lib)), ctypes.byref(g), 99, 0, ctypes.byref(h)) < 0
    del keep


def test_entry_points_reject_null_plan(lib):
    assert lib.LIB.green_gw_polarization(None, None, None, None, None, None) == -1
    assert lib.LIB.green_gw_screen(None, None, None, None, None) == -1
    assert lib.LIB.green_gw_selfenergy(None, None, None, None, None, None, None) == -1
    mu = ctypes.c_double(0.0)
    assert lib.LIB.green_dyson(None, None, None, None, None, -1.0, ctypes.byref(mu), None, None, None, None,
                               None) == -1
    rep = lib.Report()
    assert lib.LIB.green_gw_iterate(None, None, None, None, None, None, None, ctypes.byref(mu), 1.0, 1.0,
                                    ctypes.byref(rep), None, None) == -1
    assert lib.LIB.green_workspace_bytes(None) == 0
    lib.LIB.green_plan_destroy(None)


def test_build_info_names_the_sources_beside_the_library(lib):
    """The library records the digest of the sources it was built from; the binding loaded it, so the digest
    equals that of the sources in the tree, and a different digest is refused."""
    from paper_2406_18479_amd import build
    info = dict(kv.split("=", 1) for kv in lib.BUILD_INFO.split())
    assert info["sources"] == build.source_digest()
    assert info["arch"] == "gfx950"
    assert re.fullmatch(r"\d+\.\d+", info["hip"])
    saved = lib.BUILD_INFO
    try:
        lib.BUILD_INFO = saved.replace(info["sources"], "0" * 16)
        with pytest.raises(ImportError, match="other sources"):
            lib._check_provenance()
    finally:
        lib.BUILD_INFO = saved
