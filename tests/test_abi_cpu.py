"""The C ABI without a GPU: the library loads, exports every function that
include/rbc.h declares, and its host-side validation answers with the
documented status codes (no device call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rbc.h")

EINVAL = -1


@pytest.fixture(scope="module")
def lib():
    from paper_1103_2635_amd import build

    if not os.path.exists(build.LIB):
        build.build(verbose=False)
    L = ctypes.CDLL(build.LIB)
    L.rbc_last_error.restype = ctypes.c_char_p
    return L


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b((?:rbc|bf)_\w+)\s*\(", src, re.M)))


def test_every_declared_function_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 19
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, "not exported: %s" % missing


def _bf_ws(lib, m, n, d, ldq, ldx, metric, k):
    sz = ctypes.c_size_t(0)
    rc = lib.bf_search_workspace_size(ctypes.c_int64(m), ctypes.c_int64(n), ctypes.c_int32(d),
                                      ctypes.c_int64(ldq), ctypes.c_int64(ldx),
                                      ctypes.c_int32(metric), ctypes.c_int32(k), None,
                                      ctypes.byref(sz))
    return rc, sz.value


def test_bf_workspace_size_and_validation(lib):
    rc, sz = _bf_ws(lib, 1000, 5000, 64, 64, 64, 0, 1)
    assert rc == 0 and sz > 0
    # larger batches never need less workspace
    rc2, sz2 = _bf_ws(lib, 4000, 5000, 64, 64, 64, 0, 1)
    assert rc2 == 0 and sz2 >= sz
    for args, msg in [((10, 5, 8, 8, 8, 0, 10), b"exceeds"),   # k > n
                      ((10, 50, 0, 8, 8, 0, 1), None),           # d < 1
                      ((10, 50, 8, 4, 8, 0, 1), None),           # ldq < d
                      ((10, 50, 8, 8, 4, 0, 1), None),           # ldx < d
                      ((10, 50, 8, 8, 8, 7, 1), None),           # unknown metric
                      ((10, 50, 8, 8, 8, 0, 0), None)]:          # k < 1
        rc, _ = _bf_ws(lib, *args)
        assert rc == EINVAL, args
        err = lib.rbc_last_error()
        assert err and (msg is None or msg in err)


def test_autotune_set_validation(lib):
    assert lib.rbc_autotune_set(1, 64, 4, 32, 512, 0, 64) == 0
    assert lib.rbc_autotune_set(0, 128, 16, 16, 1024, 4, 64) == 0
    assert lib.rbc_autotune_set(1, 64, 4, 16, 1024, 2, 32) == 0
    for args in [(2, 64, 4, 16, 512, 0, 64), (1, 0, 4, 16, 512, 0, 64),
                 (1, 129, 4, 16, 512, 0, 64), (1, 64, 5, 16, 512, 0, 64),
                 (1, 64, 4, 24, 512, 0, 64), (1, 64, 4, 16, 0, 0, 64),
                 (1, 64, 4, 16, 512, 9, 64), (1, 64, 4, 16, 512, -1, 64),
                 (1, 64, 4, 32, 512, 0, 32), (1, 64, 4, 16, 512, 0, 48)]:
        assert lib.rbc_autotune_set(*args) == EINVAL, args
    lib.rbc_autotune_clear()


def test_free_null_is_noop(lib):
    lib.rbc_free.restype = None
    lib.rbc_free(None)
