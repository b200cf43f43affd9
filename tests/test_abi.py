"""The C ABI library loads and exports every function include/dect.h declares;
the binding refuses to run without it.  No GPU compute is called here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dect.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(dect_[a-z_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dect_project", "dect_backproject", "dect_decompose_rays",
                     "dect_admm_iterate", "dect_admm_init", "dect_plan_create"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1905_00934_amd import dect
    if not os.path.exists(dect.LIB_PATH):
        pytest.fail("libdect.so is not built; run paper_1905_00934_amd/build.py")
    lib = ctypes.CDLL(dect.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_fails_loudly_without_library(monkeypatch):
    from paper_1905_00934_amd import dect
    monkeypatch.setattr(dect, "_lib", None)
    monkeypatch.setattr(dect, "LIB_PATH", "/nonexistent/libdect.so")
    with pytest.raises(RuntimeError, match="missing"):
        dect.lib()


def test_error_message_is_thread_local_string():
    from paper_1905_00934_amd import dect
    L = dect.lib()
    # A null-argument call fails before touching the device.
    st = L.dect_plan_create(None, None, 0, None)
    assert st == -1
    assert b"null" in L.dect_last_error()
