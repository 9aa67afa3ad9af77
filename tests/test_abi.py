"""The C-ABI library loads and exports every entry point that include/kchol.h declares (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1706_02205_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "kchol.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(kc_[a-z_0-9A-Z]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_binding():
    assert set(declared_functions()) == set(_lib.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing


def test_status_strings():
    L = _lib.load()
    for s in range(7):
        assert L.kc_status_string(s)
    assert L.kc_status_string(99) == b"unknown status"


def test_invalid_arguments_are_rejected():
    import paper_1706_02205_amd as K
    x = np.random.default_rng(0).random((10, 2))
    for bad in (dict(rho=0.0), dict(rho=-1.0), dict(rho=float("nan")), dict(rho=float("inf"))):
        with pytest.raises(K.KCholError, match="invalid argument"):
            K.analyze(x, **bad)
    y = x.copy()
    y[3, 1] = np.nan
    with pytest.raises(K.KCholError, match="non-finite"):
        K.analyze(y, 2.0)
    with pytest.raises(K.KCholError):
        K.analyze(np.zeros((0, 2)), 2.0)
    with pytest.raises(ValueError):
        K.analyze(np.zeros(5), 2.0)
    L = _lib.load()
    h = C.c_void_p()
    assert L.kc_analyze(C.c_void_p(x.ctypes.data), 10, 2, 2.0, 7, 0, C.byref(h)) == _lib.KC_EINVAL
    assert L.kc_analyze(None, 10, 2, 2.0, 0, 0, C.byref(h)) == _lib.KC_EINVAL
    # factor-level calls reject a missing factor before touching a device
    w, pm, o = C.c_int32(), C.c_int64(), C.c_int()
    assert L.kc_factor_set_schedule(None, 1, 0, _lib.KC_ORDER_SPATIAL) == _lib.KC_EINVAL
    assert L.kc_factor_schedule(None, C.byref(w), C.byref(pm), C.byref(o)) == _lib.KC_EINVAL
    assert L.kc_factorize_solve(None, None, _lib.kc_kernel(0.5, 0.1), None, _lib.KC_PIVOT_ZERO, 0.0, None, None, 1,
                                None, 0, None) == _lib.KC_EINVAL
