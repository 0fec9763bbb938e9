"""C-ABI library checks that need no GPU: exports and descriptor validation.

Validation runs before any HIP call, so every invalid descriptor below is
rejected on a machine without a GPU.
"""
import ctypes
import os
import re

import pytest

from paper_2301_01145_amd import _lib, make_desc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hipoisson.h")


def header_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"HP_API\s+[\w\s\*]+?\b(hp_\w+)\s*\(", text)))


def test_library_exports_every_header_function():
    names = header_functions()
    assert len(names) == 21
    L = ctypes.CDLL(_lib.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert sorted(_lib.EXPORTS) == names


def create_status(desc):
    out = ctypes.c_void_p()
    return _lib.lib().hp_plan_create(ctypes.byref(desc), None, ctypes.byref(out))


BAD = [
    (dict(bc="dirichlet", grid="regular", nc=[8], kernel="ps", inhomogeneous=True), _lib.HP_E_UNSUPPORTED),
    (dict(bc="periodic", grid="regular", nc=[8], inhomogeneous=True, kernel="fd2"), _lib.HP_E_ARG),
    (dict(bc="periodic", grid="regular", nc=[8], diff="curl"), _lib.HP_E_ARG),
    (dict(bc="unbounded", grid="staggered", nc=[8, 8, 8], diff="curl", ncomp=1), _lib.HP_E_ARG),
    (dict(bc="periodic", grid="regular", nc=[8, 8, 8], diff="grad", ncomp=3), _lib.HP_E_ARG),
    (dict(bc="unbounded", grid="staggered", nc=[8, 8, 8], diff="div", ncomp=1), _lib.HP_E_ARG),
    (dict(bc="periodic", grid="regular", nc=[8, 8], diff="div"), _lib.HP_E_ARG),
    (dict(bc="neumann", grid="staggered", nc=[8, 8, 8], diff="nabla"), None),  # valid
    (dict(bc="neumann", grid="staggered", nc=[8, 8], diff="nabla", kernel="fd2", inhomogeneous=True),
     _lib.HP_E_UNSUPPORTED),
    (dict(bc="dirichlet", grid="regular", nc=[8, 8, 8], diff="div", ncomp=1), _lib.HP_E_ARG),
    (dict(bc="unbounded", grid="staggered", nc=[8, 8, 8], kernel="ps"), _lib.HP_E_ARG),
    (dict(bc="dirichlet", grid="staggered", nc=[8, 8, 8], kernel="spectral"), _lib.HP_E_ARG),
    (dict(bc="unbounded", grid="staggered", nc=[8], kernel="g6"), None),  # 1D order 6: valid
    (dict(bc="unbounded", grid="staggered", nc=[8, 8, 8], diff="curl", ncomp=1), _lib.HP_E_ARG),
    (dict(bc="unbounded", grid="staggered", nc=[8, 8, 8], kernel="ps"), _lib.HP_E_ARG),
    (dict(bc="dirichlet", grid="staggered", nc=[8, 8, 8], kernel="g2"), _lib.HP_E_ARG),
    (dict(bc="dirichlet", grid="staggered", nc=[8, 8, 8], diff="grad"), None),  # homogeneous: valid
    (dict(bc="dirichlet", grid="staggered", nc=[8, 8, 8], diff="curl", ncomp=3), None),  # valid
    (dict(bc="dirichlet", grid="staggered", nc=[8, 8, 8], diff="curl", ncomp=3, kernel="fd2",
          inhomogeneous=True), None),  # FD2 differences with boundary values
    (dict(bc="dirichlet", grid="staggered", nc=[8, 8], diff="grad", kernel="fd2", inhomogeneous=True), None),
    (dict(bc="neumann", grid="regular", nc=[8, 8], diff="nabla", kernel="fd2", inhomogeneous=True),
     _lib.HP_E_UNSUPPORTED),
    (dict(bc="neumann", grid="regular", nc=[1], diff="grad"), _lib.HP_E_ARG),
    (dict(bc="periodic", grid="staggered", nc=[7, 8]), None),  # prime length: a direct radix-7 stage
    # a condition per axis (HP_MIXED)
    (dict(bc=["periodic", "dirichlet"], grid="staggered", nc=[8, 8]), None),
    (dict(bc=["periodic", "unbounded"], grid="staggered", nc=[8, 8]), None),  # semi-unbounded
    (dict(bc=["unbounded", "unbounded"], grid="staggered", nc=[8, 8]), _lib.HP_E_ARG),
    (dict(bc=["unbounded", "unbounded", "neumann"], grid="staggered", nc=[8, 8, 8]), _lib.HP_E_UNSUPPORTED),
    (dict(bc=["periodic", "neumann"], grid="staggered", nc=[8, 8], diff="grad"), None),
    (dict(bc=["periodic", "unbounded"], grid="staggered", nc=[8, 8], diff="grad"), None),
    (dict(bc=["periodic", "unbounded"], grid="staggered", nc=[8, 8], diff="nabla"), _lib.HP_E_UNSUPPORTED),
    (dict(bc=["dirichlet", "unbounded"], grid="staggered", nc=[8, 8], diff="grad", kernel="fd2",
          inhomogeneous=True), _lib.HP_E_UNSUPPORTED),
    (dict(bc=["dirichlet", "neumann"], grid="staggered", nc=[8, 8], kernel="ps", inhomogeneous=True),
     _lib.HP_E_UNSUPPORTED),
    (dict(bc=["periodic", "periodic"], grid="staggered", nc=[8, 8], kernel="fd2", inhomogeneous=True),
     _lib.HP_E_ARG),  # no face takes boundary values
    (dict(bc=["neumann", "periodic"], grid="regular", nc=[8, 8], kernel="g2"), _lib.HP_E_ARG),
    (dict(bc="periodic", grid="staggered", nc=[8193], prec="f32"), _lib.HP_E_UNSUPPORTED),  # longer than a tile
    (dict(bc="periodic", grid="staggered", nc=[4097], prec="f64"), _lib.HP_E_UNSUPPORTED),
    (dict(bc="unbounded", grid="staggered", nc=[2049, 8], prec="f32"), _lib.HP_E_UNSUPPORTED),  # FP64 Green's
    (dict(bc="periodic", grid="staggered", nc=[0, 8]), _lib.HP_E_ARG),
    (dict(bc="dirichlet", grid="regular", nc=[1]), _lib.HP_E_ARG),
    (dict(bc="periodic", grid="staggered", nc=[8], lo=[1.0], hi=[1.0]), _lib.HP_E_ARG),
    (dict(bc="periodic", grid="staggered", nc=[8], ncomp=3), _lib.HP_E_ARG),
    (dict(bc="dirichlet", grid="regular", nc=[128]), None),  # 127 unknowns -> DST-I 256: valid
]


@pytest.mark.parametrize("kw,status", BAD)
def test_descriptor_validation(kw, status):
    if status is None:
        pytest.skip("valid descriptor: needs a GPU to build the plan")
    d = make_desc(**kw)
    assert create_status(d) == status
    assert _lib.hp_last_error(None) != ""


def test_bad_enum_values():
    d = make_desc("periodic", "regular", [8])
    for field, val in [("bc", 7), ("grid", 5), ("kernel", 9), ("diff", 5), ("prec", 3), ("ndim", 4), ("ncomp", 2)]:
        old = getattr(d, field)
        setattr(d, field, val)
        assert create_status(d) == _lib.HP_E_ARG, field
        setattr(d, field, old)


def test_null_arguments():
    L = _lib.lib()
    out = ctypes.c_void_p()
    assert L.hp_plan_create(None, None, ctypes.byref(out)) == _lib.HP_E_ARG
    d = make_desc("periodic", "regular", [8])
    assert L.hp_plan_create(ctypes.byref(d), None, None) == _lib.HP_E_ARG
    assert L.hp_solve(None) == _lib.HP_E_ARG
    assert L.hp_plan_destroy(None) == _lib.HP_E_ARG
    assert L.hp_query(None, 1, None) == _lib.HP_E_ARG
    s = (ctypes.c_int64 * 3)()
    assert L.hp_input_shape(None, 0, s) == _lib.HP_E_ARG


def test_status_strings():
    assert _lib.hp_status_string(0) == "ok"
    assert _lib.hp_status_string(-2) == "unsupported"
    assert _lib.hp_status_string(-9) == "unknown status"


def test_batched_validation():
    a = make_desc("neumann", "staggered", [8, 8, 8])
    b = make_desc("dirichlet", "staggered", [8, 8, 8])
    out = ctypes.c_void_p()
    arr = (_lib.hp_desc * 2)(a, b)
    assert _lib.lib().hp_plan_create_batched(arr, 2, None, ctypes.byref(out)) == _lib.HP_E_ARG
    c = make_desc("periodic", "staggered", [8, 8, 8])
    arr = (_lib.hp_desc * 1)(c)
    assert _lib.lib().hp_plan_create_batched(arr, 1, None, ctypes.byref(out)) == _lib.HP_E_UNSUPPORTED
    assert _lib.lib().hp_plan_create_batched(arr, 0, None, ctypes.byref(out)) == _lib.HP_E_ARG
    # a Dirichlet / Neumann gradient is valid for a single plan, not for a batch
    d = make_desc("neumann", "staggered", [8, 8, 8], diff="grad")
    arr = (_lib.hp_desc * 1)(d)
    assert _lib.lib().hp_plan_create_batched(arr, 1, None, ctypes.byref(out)) == _lib.HP_E_UNSUPPORTED
    assert "derivatives" in _lib.hp_last_error(None)
