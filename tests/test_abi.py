"""The C ABI: the library loads, exports every declared entry point, and its
host-side argument checks reject bad input before touching the GPU (CPU only)."""
import ctypes as C
import os
import re

import pytest

from paper_2402_18008_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "homog.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_abi.LIB_PATH):
        from paper_2402_18008_amd import build
        build.build()
    return _abi.lib()


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hg_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding declares a signature for each of them
    assert set(names) <= set(_abi.SIGNATURES)


def test_status_strings(lib):
    assert lib.hg_version() >= 10000
    for st in (0, -1, -2, -3, -4):
        assert lib.hg_status_str(st)


FAKE = C.c_void_p(0x1000)   # never dereferenced: validation fails first


def test_solve4_validation(lib):
    f = lib.hg_solve4
    assert f(7, FAKE, FAKE, 10, 10, FAKE, None, None) == _abi.HG_EINVAL
    assert b"method" in lib.hg_last_error()
    assert f(0, FAKE, FAKE, -1, 10, FAKE, None, None) == _abi.HG_EINVAL
    assert f(0, FAKE, FAKE, 10, 9, FAKE, None, None) == _abi.HG_EINVAL
    assert f(0, None, FAKE, 10, 10, FAKE, None, None) == _abi.HG_EINVAL
    assert f(0, FAKE, FAKE, 10, 10, None, None, None) == _abi.HG_EINVAL
    # n == 0 is a no-op even with NULL pointers
    assert f(0, None, None, 0, 0, None, None, None) == _abi.HG_OK
    assert f(1, None, None, 0, 0, None, None, None) == _abi.HG_OK
