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
    assert L.hsgn_set_launch(None, 1) == -1
    L.hsgn_set_halo_margin.argtypes = [ctypes.c_void_p, ctypes.c_double]
    assert L.hsgn_set_halo_margin(None, 1.0) == -1
    assert L.hsgn_autotune_launch(None, 1, None, None) == -1
    assert L.hsgn_set_halo_retry(None, 1) == -1
    L.hsgn_set_adjoint_tape_bytes.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    assert L.hsgn_set_adjoint_tape_bytes(None, 0) == -1
    assert L.hsgn_halo_state(None, None, None) == -1
    L.hsgn_destroy(None)


def test_binding_refuses_to_run_without_the_library(monkeypatch, tmp_path):
    import paper_2510_07539_amd.hsgn as H
    monkeypatch.setattr(H, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(H, "_lib", None)
    import pytest
    with pytest.raises(RuntimeError):
        H.lib()


def test_init_rejects_invalid_parameters_without_a_device():
    """hsgn_init validates every instance before its first HIP call: each
    invalid set below returns HSGN_EINVAL (-1) and leaves no context."""
    from paper_2510_07539_amd.hsgn import HsgnParams
    L = ctypes.CDLL(LIB)
    L.hsgn_init.restype = ctypes.c_int
    L.hsgn_init.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                            ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(HsgnParams),
                            ctypes.c_void_p, ctypes.c_void_p]

    def good():
        return dict(g=9.81, lam=100.0, dx=0.25, cfl=0.9, mcfl=0.5, dt_fixed=0.0, t_end=0.0,
                    bc=1, has_bathymetry=0, order=2, scheme=0)

    def init(sizes, changes, d_b=None, first=0):
        offs = [first]
        for n in sizes:
            offs.append(offs[-1] + n)
        off = (ctypes.c_int64 * len(offs))(*offs)
        ps = (HsgnParams * len(sizes))()
        for j in range(len(sizes)):
            kw = good()
            kw.update(changes[j] if j < len(changes) else {})
            ps[j] = HsgnParams(**kw)
        h = ctypes.c_void_p()
        rc = L.hsgn_init(ctypes.byref(h), len(sizes), off, ps, d_b, None)
        return rc, h.value

    fake_bed = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    cases = [
        ([3], [{}]),                                   # fewer than 4 cells
        ([8], [{"bc": 2}]),                            # unknown boundary type
        ([8], [{"lam": 0.0}]),                         # lambda must be positive
        ([8], [{"g": -9.81}]),                         # gravity must be positive
        ([8], [{"dx": 0.0}]),                          # cell width must be positive
        ([8], [{"cfl": 0.0}]),                         # no CFL and no fixed step
        ([8], [{"has_bathymetry": 1}]),                # bed without a bed array
        ([8], [{"order": 3}]),                         # unknown order
        ([8, 8], [{}, {"order": 1}]),                  # order differs between instances
        ([8], [{"scheme": 3}]),                        # unknown scheme
        ([8, 8], [{}, {"scheme": 1}]),                 # scheme differs between instances
        ([8], [{"scheme": 2, "order": 1}]),            # SGN with the first-order step
    ]
    for sizes, changes in cases:
        rc, h = init(sizes, changes)
        assert rc == -1, (sizes, changes, rc)
        assert not h
    rc, h = init([8], [{"scheme": 1, "has_bathymetry": 1}], d_b=fake_bed)  # explicit over a bed
    assert rc == -1 and not h
    rc, h = init([8], [{}], first=1)                   # offsets must start at 0
    assert rc == -1 and not h
