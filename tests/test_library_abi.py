"""CPU-side checks of the C ABI: the library loads and exports every entry
point that include/semx.h declares (no GPU call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    txt = open(os.path.join(ROOT, "include", header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(semx_[a-z0-9_]+)\s*\(", txt)))


def _lib():
    import paper_2606_12850_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.fail("libsemx.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(P.LIB_PATH)


def test_header_declares_entry_points():
    names = _declared("semx.h")
    for must in ["semx_create", "semx_destroy", "semx_upload_mesh", "semx_upload_model",
                 "semx_apply_force", "semx_step", "semx_read_seismograms"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    L = _lib()
    missing = [n for n in _declared("semx.h") if getattr(L, n, None) is None]
    assert not missing, missing


def test_binding_wraps_every_declared_symbol():
    import paper_2606_12850_amd as P
    names = _declared("semx.h")
    missing = [n for n in names if not hasattr(P, n)]
    assert not missing, missing
    assert set(names) <= set(P.exported_symbols())


def test_create_rejects_bad_ngll_without_gpu():
    # argument validation happens before any HIP call
    import paper_2606_12850_amd as P
    h = ctypes.c_void_p()
    assert P.lib().semx_create(ctypes.byref(h), 1, None) == P.SEMX_EINVAL
    assert P.lib().semx_create(ctypes.byref(h), 17, None) == P.SEMX_EINVAL
    assert P.lib().semx_create(None, 5, None) == P.SEMX_EINVAL
    assert P.lib().semx_destroy(None) == P.SEMX_OK


def test_gll_query_without_gpu():
    # semx_gll makes no HIP call: nodes and weights agree with the oracle's
    import numpy as np
    import paper_2606_12850_amd as P
    from oracle import oracle as O
    for n in (2, 5, 16):
        xi, w = P.semx_gll(n)
        xo, wo = O.gll(n)
        np.testing.assert_allclose(xi, xo, atol=1e-15)
        np.testing.assert_allclose(w, wo, atol=1e-15)
    for bad in (1, 17):
        assert P.lib().semx_gll(bad, None, None) == P.SEMX_EINVAL
