"""The C ABI: the library loads, exports every function include/dgns.h declares,
and rejects bad arguments before touching the GPU (CPU only)."""
import ctypes
import os
import re

import pytest

import paper_1806_03095_amd as pkg
from paper_1806_03095_amd import binding

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "dgns.h")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(dgns_\w+)\s*\(", src, re.M)))


def test_header_and_binding_agree():
    assert declared() == sorted(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = pkg.load_library()
    for name in declared():
        assert hasattr(lib, name), name


def _params(**kw):
    p = binding.Params(3, 6, 0, 0, 1.4, 287.0, 1e-3, 1.0, 1.0, (ctypes.c_double * 3)(0, 0, 0), 0.0)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _mesh(**kw):
    m = binding.BoxMesh((ctypes.c_int * 3)(2, 2, 2), (ctypes.c_double * 3)(0, 0, 0), (ctypes.c_double * 3)(1, 1, 1),
                        (ctypes.c_int * 3)(1, 1, 1), 0, 1.8, 0.0)
    for k, v in kw.items():
        setattr(m, k, v)
    return m


@pytest.mark.parametrize("pkw,mkw,code", [
    (dict(degree=0), {}, binding.EINVAL),
    (dict(degree=16), {}, binding.EINVAL),
    (dict(n_q=0), {}, binding.EINVAL),
    (dict(n_q=17), {}, binding.EINVAL),
    (dict(n_q=10), {}, binding.EUNSUPPORTED),
    (dict(degree=8, n_q=12), {}, binding.EUNSUPPORTED),
    (dict(degree=8, n_q=9, body_force=(ctypes.c_double * 3)(1, 0, 0)), {}, binding.EUNSUPPORTED),
    (dict(basis=5), {}, binding.EINVAL),
    (dict(precision=3), {}, binding.EINVAL),
    (dict(gamma=1.0), {}, binding.EINVAL),
    (dict(mu=-1.0), {}, binding.EINVAL),
    ({}, dict(kind=7), binding.EINVAL),
    ({}, dict(n=(ctypes.c_int * 3)(0, 2, 2)), binding.EINVAL),
    ({}, dict(hi=(ctypes.c_double * 3)(0, 1, 1)), binding.EINVAL),
    ({}, dict(periodic=(ctypes.c_int * 3)(1, 0, 1)), binding.EINVAL),   # walls without wall_T
])
def test_create_rejects_bad_arguments(pkw, mkw, code):
    lib = pkg.load_library()
    h = ctypes.c_void_p(123)
    rc = lib.dgns_create(ctypes.byref(_params(**pkw)), ctypes.byref(_mesh(**mkw)), None, ctypes.byref(h))
    assert rc == code
    assert h.value is None
    assert len(lib.dgns_last_error()) > 0


def test_null_arguments():
    lib = pkg.load_library()
    assert lib.dgns_create(None, None, None, None) == binding.EINVAL
    assert lib.dgns_sizes(None, None, None, None) == binding.EINVAL
    assert lib.dgns_apply_operator(None, None, None, 0.0) == binding.EINVAL
    assert lib.dgns_rk_step(None, None, None, 0.0, 0.1) == binding.EINVAL
    assert lib.dgns_rk_stage_update(None, None, None, None, 0, 0.1) == binding.EINVAL
    assert lib.dgns_channel_statistics(None, None, None) == binding.EINVAL
    assert lib.dgns_destroy(None) == binding.OK
    assert b"null" in lib.dgns_last_error() or len(lib.dgns_last_error()) > 0
