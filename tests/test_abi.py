"""The C-ABI library builds for gfx950, loads on the host and exports every
function that include/hsgn.h declares (no compute calls: no GPU here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "hsgn.h")
LIB = os.path.join(ROOT, "paper_2510_07539_amd", "libhsgn.so")


def declared():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hsgn_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for need in ("hsgn_init", "hsgn_step", "hsgn_run", "hsgn_adjoint", "hsgn_set_state",
                 "hsgn_get_state", "hsgn_status", "hsgn_last_error", "hsgn_destroy"):
        assert need in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        from paper_2510_07539_amd import build
        build.build()
    L = ctypes.CDLL(LIB)
    for name in declared():
        assert hasattr(L, name), name
    L.hsgn_version.restype = ctypes.c_char_p
    assert L.hsgn_version().startswith(b"hsgn-gfx950")


def test_null_arguments_are_rejected_without_a_device():
    L = ctypes.CDLL(LIB)
    L.hsgn_init.restype = ctypes.c_int
    assert L.hsgn_init(None, 1, None, None, None, None) == -1
    h = ctypes.c_void_p()
    assert L.hsgn_init(ctypes.byref(h), 0, None, None, None, None) == -1
    assert L.hsgn_step(None, 1) == -1
    assert L.hsgn_run(None, 1, 2) == -1
    assert L.hsgn_adjoint(None, 1, 1, 1, None, None, None, None, None, None) == -1
    assert L.hsgn_set_solver(None, 0) == -1
    L.hsgn_destroy(None)


def test_binding_refuses_to_run_without_the_library(monkeypatch, tmp_path):
    import paper_2510_07539_amd.hsgn as H
    monkeypatch.setattr(H, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(H, "_lib", None)
    import pytest
    with pytest.raises(RuntimeError):
        H.lib()
