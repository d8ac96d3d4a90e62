"""The C ABI contract, checked on the host: the built library loads, exports
every function include/isg.h declares, and rejects bad arguments before any
device work.  No compute call is made here."""
import ctypes as C
import os
import re

import pytest

from paper_2501_16713_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "isg.h")

needs_lib = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="libisg.so not built")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(isg_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert _declared() == sorted(_lib.SIGNATURES)


@needs_lib
def test_library_exports_every_declared_symbol():
    lib = C.CDLL(_lib.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


@needs_lib
def test_version_and_empty_error():
    lib = _lib.load()
    assert lib.isg_version().decode().startswith("isg")
    assert isinstance(lib.isg_last_error().decode(), str)


def _desc(ndim=3, n=(16, 16, 16), C_=2, P=1, storage=0):
    d = _lib.isg_plan_desc()
    d.ndim = ndim
    for i, v in enumerate(n):
        d.n[i] = v
    d.ncoils = C_
    d.nphases = P
    d.storage = storage
    d.stream = None
    return d


@needs_lib
@pytest.mark.parametrize("kw,status", [
    (dict(ndim=4), 1),
    (dict(C_=0), 1),
    (dict(C_=33), 1),
    (dict(P=0), 1),
    (dict(storage=7), 1),
    (dict(n=(16, 14, 16)), 2),   # prime factor 7
    (dict(n=(16, 15, 16)), 2),   # odd
    (dict(n=(6, 16, 16)), 2),    # too small
    (dict(n=(1024, 16, 16)), 2), # too large
    (dict(n=(16, 16, 512), C_=16), 2),  # coils x 2 n_last > 8192
])
def test_plan_create_validation(kw, status):
    lib = _lib.load()
    h = C.c_void_p()
    d = _desc(**kw)
    assert lib.isg_plan_create(C.byref(d), C.byref(h)) == status
    assert not h.value
    assert lib.isg_last_error().decode()


@needs_lib
def test_null_arguments():
    lib = _lib.load()
    h = C.c_void_p()
    assert lib.isg_plan_create(None, C.byref(h)) == 1
    assert lib.isg_warp(None, None, None, None) == 1
    assert lib.isg_normal(None, 1, None, 0.0, None, None, None, None) == 1
    assert lib.isg_plan_destroy(None) == 0
    assert lib.isg_motion_destroy(None) == 0
    assert lib.isg_traj_destroy(None) == 0
    cnt = C.c_int(-1)
    assert lib.isg_device_count(C.byref(cnt)) == 0 and cnt.value >= 0


@needs_lib
def test_no_device_reports_device_error():
    lib = _lib.load()
    cnt = C.c_int(0)
    lib.isg_device_count(C.byref(cnt))
    if cnt.value > 0:
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    d = _desc()
    assert lib.isg_plan_create(C.byref(d), C.byref(h)) == 4
    assert "device" in lib.isg_last_error().decode().lower()


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        _lib.load(str(tmp_path / "nope.so"))
