"""Host-side checks of the C ABI (no GPU needed): the library loads and exports
every entry point include/grating.h declares, and argument errors are reported."""
import ctypes as C
import os
import subprocess

import pytest

from paper_1412_7466_amd import grating

LIB = grating.LIB_PATH


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libgrating.so is not built (run python -m paper_1412_7466_amd.build)")
    return grating.load_library()


def test_header_symbols_exported(lib):
    names = grating.exported_symbols()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    for n in names:
        assert f" T {n}\n" in out or f" T {n}" in out, n


def test_binding_covers_header():
    assert set(grating.exported_symbols()) == set(grating._PROTOS)


def test_null_context_rejected(lib):
    assert lib.grt_build(None) == grating.GRT_EINVAL
    assert lib.grt_apply(None, None, None, 0) == grating.GRT_EINVAL
    assert lib.grt_create(None, 0, None) == grating.GRT_EINVAL
    assert lib.grt_error_message(None) == b"null context"


def test_noalloc_rejects_bad_arguments_on_host(lib):
    """grt_apply_T_noalloc checks its arguments before touching a device."""
    f = lib.grt_apply_T_noalloc
    p = C.c_void_p(16)   # never dereferenced: every call below fails its host checks
    ok = dict(M=4, P=10, k2=10.0, d=1.0, ar=1.0, ai=0.0)

    def call(**kw):
        a = {**ok, **kw}
        return f(a["M"], a["P"], a["k2"], a["d"], a["ar"], a["ai"], p, p, p, C.c_void_p(32), None)

    assert call(M=0) == grating.GRT_EINVAL
    assert call(k2=-1.0) == grating.GRT_EINVAL
    assert call(ar=2.0) == grating.GRT_EINVAL              # |alpha| must be 1
    assert call(P=7) == grating.GRT_EUNSUP                 # P not compiled in
    assert call(M=200_000, P=20) == grating.GRT_EINVAL     # one partial exceeds the scratch
    assert f(4, 10, 10.0, 1.0, 1.0, 0.0, None, p, p, C.c_void_p(32), None) == grating.GRT_EINVAL
    assert f(4, 10, 10.0, 1.0, 1.0, 0.0, p, p, p, p, None) == grating.GRT_EINVAL   # x aliases y
