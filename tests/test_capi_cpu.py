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
