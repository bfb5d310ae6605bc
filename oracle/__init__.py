"""Plain FP64 CPU oracle of the semi-implicit IMEX hSGN step (arXiv 2510.07539).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  It shares no code with the HIP
library; the C source `hsgn_oracle.c` is compiled here with gcc (no
-ffast-math, no FMA contraction) into `liboracle.so`.

Python side: ctypes marshalling plus a few helpers that follow the paper's
definitions directly (no arithmetic of the scheme lives in this file).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hsgn_oracle.c")
_SRC_CS = os.path.join(_HERE, "hsgn_oracle_cs.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_CS = os.path.join(_HERE, "liboracle_cs.so")
_lib = None
_lib_cs = None

OK, ENONPHYS, ENONCOERCIVE, EINVAL = 0, 1, 2, 3
BC_PERIODIC, BC_TRANSMISSIVE = 0, 1


# gcc flags of both builds: portable code, no FMA contraction, no fast math,
# OpenMP over instances
COMPILE_FLAGS = ["-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                 "-fno-fast-math", "-Wall", "-Wno-unused-label"]


def _compile(src, lib):
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = ["gcc", *COMPILE_FLAGS, src, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, lib)


def _stale(lib):
    return (not os.path.exists(lib)) or os.path.getmtime(lib) < max(
        os.path.getmtime(_SRC), os.path.getmtime(_SRC_CS))


def build(force: bool = True) -> str:
    """Compile liboracle.so and its complex-step twin liboracle_cs.so with gcc
    (portable flags, no FMA contraction, OpenMP over instances)."""
    for src, lib in ((_SRC, _LIB), (_SRC_CS, _LIB_CS)):
        if force or _stale(lib):
            _compile(src, lib)
    return _LIB


class Params(C.Structure):
    _fields_ = [("g", C.c_double), ("lam", C.c_double), ("dx", C.c_double),
                ("cfl", C.c_double), ("mcfl", C.c_double), ("dt_fixed", C.c_double),
                ("t_end", C.c_double), ("bc", C.c_int), ("has_b", C.c_int),
                ("order", C.c_int), ("scheme", C.c_int), ("form", C.c_int)]


class StageDbg(C.Structure):
    _fields_ = [(k, C.POINTER(C.c_double)) for k in
                ("qd", "md", "Wd", "beta", "S", "phi", "T", "P0", "pt0",
                 "lo", "di", "up", "rhs", "hbar", "Fq", "Fm", "FW")]


def lib():
    global _lib
    if _lib is None:
        if _stale(_LIB) or _stale(_LIB_CS):
            build(force=False)
        _lib = _configure(C.CDLL(_LIB))
    return _lib


def _configure(L):
    """Declare the argument and result types of the double build."""
    dp = C.POINTER(C.c_double)
    L.or_stage.restype = C.c_int
    L.or_stage.argtypes = [C.c_int, C.POINTER(Params), C.c_double, dp] + [dp] * 12 + [C.POINTER(StageDbg)]
    L.or_dt.restype = C.c_double
    L.or_dt.argtypes = [C.c_int, C.POINTER(Params), dp, dp, C.c_double]
    L.or_sgn_phi.restype = C.c_int
    L.or_sgn_phi.argtypes = [C.c_int, C.POINTER(Params), dp, dp, dp]
    L.or_dt_ex.restype = C.c_double
    L.or_dt_ex.argtypes = [C.c_int, C.POINTER(Params), dp, dp, dp, C.c_double]
    L.or_step.restype = C.c_int
    L.or_step.argtypes = [C.c_int, C.POINTER(Params), dp, dp, dp, dp, dp, dp, dp]
    L.or_run.restype = C.c_int
    L.or_run.argtypes = [C.c_int, C.POINTER(Params), dp, dp, dp, dp, dp, dp, C.c_int]
    L.or_run_batch.restype = C.c_int
    L.or_run_batch.argtypes = [C.c_int, C.POINTER(C.c_longlong), C.POINTER(Params), dp,
                               dp, dp, dp, dp, dp, C.c_int, C.c_int, C.POINTER(C.c_int)]
    L.or_tridiag.restype = C.c_int
    L.or_tridiag.argtypes = [C.c_int, C.c_int, dp, dp, dp, dp, dp]
    L.or_gamma.restype = C.c_double
    L.or_max_threads.restype = C.c_int
    L.or_tableau.restype = None
    L.or_tableau.argtypes = [dp]
    ip = C.POINTER(C.c_int)
    L.or_run_loss.restype = C.c_int
    L.or_run_loss.argtypes = [C.c_int, C.POINTER(Params), dp, dp, dp, dp, dp, C.c_int,
                              C.c_int, ip, dp, dp]
    L.or_run_gauges.restype = C.c_int
    L.or_run_gauges.argtypes = [C.c_int, C.POINTER(Params), dp, dp, dp, dp, dp, C.c_int,
                                C.c_int, ip, dp]
    return L


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


SCHEME_SI, SCHEME_EXPLICIT, SCHEME_SGN = 0, 1, 2


FORM_P, FORM_A = 0, 1


def make_params(g=9.81, lam=100.0, dx=1.0, cfl=0.9, mcfl=0.5, dt_fixed=0.0,
                t_end=0.0, bc=BC_PERIODIC, has_b=0, order=2, scheme=SCHEME_SI,
                form=FORM_P) -> Params:
    """form: FORM_P (conservative P-form, the oracle of the library) or
    FORM_A (the printed lines of Sec. 4.2, CPU only, flat bottom)."""
    return Params(g, lam, dx, cfl, mcfl, dt_fixed, t_end, int(bc), int(has_b), int(order),
                  int(scheme), int(form))


def gamma() -> float:
    return lib().or_gamma()


def tableau():
    """(gamma, 1 - c/gamma, c/gamma, 1 - (1-gamma)/gamma, (1-gamma)/gamma) as used."""
    out = np.empty(5)
    lib().or_tableau(_p(out))
    return tuple(out)


def max_threads() -> int:
    return lib().or_max_threads()


def _f(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def stage(p: Params, tau, b, UE, Uold, debug=False):
    """One semi-implicit stage.  UE, Uold: 4-tuples (h, q, m, W).
    Returns (rc, Unew[, dbg dict])."""
    n = len(UE[0])
    UE = [_f(a) for a in UE]
    Uo = [_f(a) for a in Uold]
    out = [np.empty(n) for _ in range(4)]
    bb = _f(b) if b is not None else None
    dbg = None
    arrays = {}
    if debug:
        for k, _ in StageDbg._fields_:
            arrays[k] = np.empty(n + 1 if k in ("Fq", "Fm", "FW") else n)
        dbg = StageDbg(**{k: _p(v) for k, v in arrays.items()})
    rc = lib().or_stage(n, C.byref(p), float(tau), _p(bb), *[_p(a) for a in UE],
                        *[_p(a) for a in Uo], *[_p(a) for a in out],
                        C.byref(dbg) if dbg is not None else None)
    if debug:
        return rc, tuple(out), arrays
    return rc, tuple(out)


def dt(p: Params, h, q, t=0.0) -> float:
    h, q = _f(h), _f(q)
    return lib().or_dt(len(h), C.byref(p), _p(h), _p(q), float(t))


def dt_ex(p: Params, h, q, m, t=0.0) -> float:
    h, q, m = _f(h), _f(q), _f(m)
    return lib().or_dt_ex(len(h), C.byref(p), _p(h), _p(q), _p(m), float(t))


def sgn_phi(p: Params, h, q):
    """phi of the standard SGN elliptic problem; returns (rc, phi)."""
    h, q = _f(h), _f(q)
    phi = np.empty(len(h))
    rc = lib().or_sgn_phi(len(h), C.byref(p), _p(h), _p(q), _p(phi))
    return rc, phi


def step(p: Params, b, U, t=0.0):
    """One step (scheme and order from p); returns (rc, Unew, t_new, dt)."""
    U = [np.array(a, dtype=np.float64, copy=True) for a in U]
    tt = C.c_double(t)
    dtt = C.c_double(0.0)
    bb = _f(b) if b is not None else None
    rc = lib().or_step(len(U[0]), C.byref(p), _p(bb), *[_p(a) for a in U],
                       C.pointer(tt), C.pointer(dtt))
    return rc, tuple(U), tt.value, dtt.value


def run(p: Params, b, U, t=0.0, nsteps=1):
    """nsteps IMEX steps; returns (rc, Unew, t_new)."""
    U = [np.array(a, dtype=np.float64, copy=True) for a in U]
    tt = C.c_double(t)
    bb = _f(b) if b is not None else None
    rc = lib().or_run(len(U[0]), C.byref(p), _p(bb), *[_p(a) for a in U],
                      C.pointer(tt), int(nsteps))
    return rc, tuple(U), tt.value


def run_batch(offsets, plist, b, U, t, nsteps, nthreads=0):
    """Batched instances (OpenMP over instances).  Returns (rc, Unew, t, status)."""
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    n_inst = len(offs) - 1
    parr = (Params * n_inst)(*plist)
    U = [np.array(a, dtype=np.float64, copy=True) for a in U]
    tt = np.array(t, dtype=np.float64, copy=True).reshape(n_inst)
    st = np.zeros(n_inst, dtype=np.int32)
    bb = _f(b) if b is not None else None
    rc = lib().or_run_batch(n_inst, offs.ctypes.data_as(C.POINTER(C.c_longlong)), parr,
                            _p(bb), *[_p(a) for a in U], _p(tt), int(nsteps), int(nthreads),
                            st.ctypes.data_as(C.POINTER(C.c_int)))
    return rc, tuple(U), tt, st


def tridiag(lo, di, up, rhs, cyclic=False):
    lo, di, up, rhs = _f(lo), _f(di), _f(up), _f(rhs)
    x = np.empty(len(di))
    rc = lib().or_tridiag(len(di), int(bool(cyclic)), _p(lo), _p(di), _p(up), _p(rhs), _p(x))
    return rc, x


def lib_cs():
    """Complex-step build: arrays are complex128 (interleaved re, im)."""
    global _lib_cs
    if _lib_cs is None:
        lib()
        _lib_cs = _configure_cs(C.CDLL(_LIB_CS))
    return _lib_cs


def _configure_cs(L):
    cp = C.c_void_p
    ip = C.POINTER(C.c_int)
    dp = C.POINTER(C.c_double)
    L.or_run_loss_cs.restype = C.c_int
    L.or_run_loss_cs.argtypes = [C.c_int, C.POINTER(Params), cp, cp, cp, cp, cp, C.c_int,
                                 C.c_int, ip, dp, cp]
    L.or_run_cs.restype = C.c_int
    L.or_run_cs.argtypes = [C.c_int, C.POINTER(Params), cp, cp, cp, cp, cp, dp, C.c_int]
    L.or_step_cs.restype = C.c_int
    L.or_step_cs.argtypes = [C.c_int, C.POINTER(Params), cp, cp, cp, cp, cp, dp, dp]
    return L


class using:
    """Context manager: the functions of this module call the oracle built
    from another copy of the source (libraries in `libdir`, built by
    `build_at`), e.g. a copy with a planted mistake, for tests that check
    that the pins detect it.  Restores the regular build on exit."""

    def __init__(self, libdir):
        self.libdir = libdir

    def __enter__(self):
        global _lib, _lib_cs
        lib()
        lib_cs()
        self.saved = (_lib, _lib_cs)
        _lib = _configure(C.CDLL(os.path.join(self.libdir, "liboracle.so")))
        _lib_cs = _configure_cs(C.CDLL(os.path.join(self.libdir, "liboracle_cs.so")))
        return self

    def __exit__(self, *exc):
        global _lib, _lib_cs
        _lib, _lib_cs = self.saved
        return False


def build_at(libdir, source_text):
    """Compile `source_text` (a variant of hsgn_oracle.c) into libdir as
    liboracle.so and liboracle_cs.so with the regular flags."""
    import shutil
    os.makedirs(libdir, exist_ok=True)
    for f in ("hsgn_oracle.h", "hsgn_oracle_cs.c"):
        shutil.copy(os.path.join(_HERE, f), os.path.join(libdir, f))
    with open(os.path.join(libdir, "hsgn_oracle.c"), "w") as f:
        f.write(source_text)
    _compile(os.path.join(libdir, "hsgn_oracle.c"), os.path.join(libdir, "liboracle.so"))
    _compile(os.path.join(libdir, "hsgn_oracle_cs.c"), os.path.join(libdir, "liboracle_cs.so"))


def source_text():
    with open(_SRC) as f:
        return f.read()


def step_jacobian(p: Params, b, U, eps=1e-30):
    """Jacobian of one step (scheme and order from p) with respect to the
    state (h, q, m, W), by complex steps of the complex build: column k is
    Im step(U + i eps e_k) / eps, exact to rounding.  Use a fixed dt
    (p.dt_fixed > 0) so that dt does not depend on the state.  Returns
    (rc, J) with J of shape (4n, 4n), fields stacked h, q, m, W."""
    n = len(U[0])
    base = np.concatenate([np.asarray(a, dtype=np.float64) for a in U])
    J = np.empty((4 * n, 4 * n))
    bb = None if b is None else np.ascontiguousarray(b, dtype=np.complex128)
    vp = lambda a: None if a is None else C.c_void_p(a.ctypes.data)
    for k in range(4 * n):
        z = base.astype(np.complex128)
        z[k] += 1j * eps
        Uc = [np.ascontiguousarray(z[f * n:(f + 1) * n]) for f in range(4)]
        t = C.c_double(0.0)
        dtt = C.c_double(0.0)
        rc = lib_cs().or_step_cs(n, C.byref(p), vp(bb), *[vp(a) for a in Uc], C.pointer(t),
                                 C.pointer(dtt))
        if rc:
            return rc, None
        J[:, k] = np.concatenate([a.imag for a in Uc]) / eps
    return 0, J


def run_loss(p: Params, b, U, nsteps, gauges, targets):
    """Gauge-misfit loss of nsteps steps (double build).  Returns (rc, J, Unew)."""
    U = [np.array(a, dtype=np.float64, copy=True) for a in U]
    g = np.ascontiguousarray(gauges, dtype=np.int32)
    tg = np.ascontiguousarray(targets, dtype=np.float64).reshape(-1)
    J = C.c_double(0.0)
    bb = _f(b) if b is not None else None
    rc = lib().or_run_loss(len(U[0]), C.byref(p), _p(bb), *[_p(a) for a in U], int(nsteps),
                           len(g), g.ctypes.data_as(C.POINTER(C.c_int)), _p(tg), C.pointer(J))
    return rc, J.value, tuple(U)


def run_gauges(p: Params, b, U, nsteps, gauges):
    """Gauge series (nsteps, n_gauge) of h after each step.  Returns (rc, series)."""
    U = [np.array(a, dtype=np.float64, copy=True) for a in U]
    g = np.ascontiguousarray(gauges, dtype=np.int32)
    out = np.zeros((int(nsteps), len(g)))
    bb = _f(b) if b is not None else None
    rc = lib().or_run_gauges(len(U[0]), C.byref(p), _p(bb), *[_p(a) for a in U], int(nsteps),
                             len(g), g.ctypes.data_as(C.POINTER(C.c_int)), _p(out))
    return rc, out


def run_loss_cs(p: Params, b, U, nsteps, gauges, targets):
    """Same on complex128 inputs (complex-step).  Returns (rc, J complex)."""
    U = [np.array(a, dtype=np.complex128, copy=True) for a in U]
    g = np.ascontiguousarray(gauges, dtype=np.int32)
    tg = np.ascontiguousarray(targets, dtype=np.float64).reshape(-1)
    J = np.zeros(1, dtype=np.complex128)
    bb = None if b is None else np.ascontiguousarray(b, dtype=np.complex128)
    vp = lambda a: None if a is None else C.c_void_p(a.ctypes.data)
    rc = lib_cs().or_run_loss_cs(len(U[0]), C.byref(p), vp(bb), *[vp(a) for a in U], int(nsteps),
                               len(g), g.ctypes.data_as(C.POINTER(C.c_int)),
                               tg.ctypes.data_as(C.POINTER(C.c_double)), vp(J))
    return rc, complex(J[0])
