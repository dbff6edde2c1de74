"""CPU checks of the C-ABI library: it loads, exports every function that
include/osc.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "osc.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-zA-Z_][a-zA-Z0-9_]*\s*\*?\s*(osc_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_1702_02207_amd import osc
    if not os.path.exists(osc.LIB_PATH):
        pytest.skip("libosc.so not built")
    return osc.load()


def test_header_declares_functions():
    names = _declared_functions()
    assert "osc_create" in names and "osc_integrate" in names and "osc_energy" in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), f"{name} declared in osc.h but not exported"


def test_abi_version(lib):
    assert lib.osc_abi_version() == 1


def test_null_arguments_rejected_without_device(lib):
    from paper_1702_02207_amd import osc
    h = ctypes.c_void_p()
    assert lib.osc_create(None, None, ctypes.byref(h)) == osc.OSC_EINVAL
    assert b"desc" in lib.osc_last_error()
    d = osc.Desc(0, 0, 1, 0, 1, 0, 0, None, None, None)      # s = 0
    assert lib.osc_create(ctypes.byref(d), None, ctypes.byref(h)) == osc.OSC_EINVAL
    d = osc.Desc(0, 7, 1, 2, 1, 0, 0, 1, 1, 1)               # bad method
    assert lib.osc_create(ctypes.byref(d), None, ctypes.byref(h)) == osc.OSC_EINVAL
    assert lib.osc_integrate(None, None, None, 1, 0, None, None, None, None) == osc.OSC_EINVAL
    assert lib.osc_energy(None, None, None, None) == osc.OSC_EINVAL
    assert lib.osc_sync(None) == osc.OSC_EINVAL
    lib.osc_destroy(None)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1702_02207_amd import osc
    monkeypatch.setattr(osc, "_lib", None)
    monkeypatch.setattr(osc, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(osc.OscError):
        osc.load()
