"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/lt.h declares, and rejects bad arguments before any
device work."""
import ctypes as C
import os
import re

import pytest

import paper_2306_06744_amd as lt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lt_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(lt.SO_PATH):
        from paper_2306_06744_amd import build
        build.build()
    return lt.lib()


def test_header_matches_binding():
    assert _declared() == sorted(lt.EXPORTS)


def test_every_declared_symbol_is_exported(L):
    for name in _declared():
        assert hasattr(L, name), name


def test_oracle_is_not_linked():
    """The product library does not depend on the oracle."""
    data = open(lt.SO_PATH, "rb").read()
    assert b"lto_" not in data and b"lt_oracle" not in data


def test_bad_geometry_rejected_on_host(L):
    h = C.c_void_p()
    g = lt.Geom(4, 0, 3, 0, 2)
    assert L.lt_build_uniform(C.byref(g), 1, None, C.byref(h)) == 1
    assert b"dim" in L.lt_last_error()
    g = lt.Geom(3, 0, 21, 7, 2)   # 3*21 + 5 bits > 64
    assert L.lt_build_uniform(C.byref(g), 1, None, C.byref(h)) == 4
    g = lt.Geom(2, 5, 3, 3, 2)    # d_min > d_max
    assert L.lt_build_uniform(C.byref(g), 1, None, C.byref(h)) == 4
    g = lt.Geom(2, 0, 6, 3, 7)    # bad balance kind
    assert L.lt_build_uniform(C.byref(g), 1, None, C.byref(h)) == 1
    assert not h.value


def test_null_tree_rejected(L):
    n = C.c_int64()
    assert L.lt_size(None, C.byref(n), None, None) == 1
    assert L.lt_balance(None, None) == 1
    assert L.lt_build(None, None, 0, None, None) == 1
    L.lt_destroy(None)  # ignored
