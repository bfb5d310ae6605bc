"""Python binding of the gfx950 hSGN library (libhsgn.so, C ABI in include/hsgn.h).

Argument marshalling only: every step of the solver runs in the HIP kernels.
PyTorch provides device memory and the stream.  If the library is not built,
importing this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhsgn.so")

HSGN_OK, HSGN_EINVAL, HSGN_EHIP, HSGN_ENONPHYS, HSGN_ENONCOERCIVE, HSGN_ENOMEM = 0, -1, -2, -3, -4, -5
HSGN_EWINDOW = -6
FLAG_NONPHYS, FLAG_NONCOERCIVE = 1, 2
KERNEL_KINDS = ("dt", "reduce1", "rsolve1", "stage1", "reduce2", "rsolve2", "stage2", "win1", "win2",
                "ex1", "ex2", "sgn_rows", "sgn_solve", "sgn_update")
SOLVER_AUTO, SOLVER_EXACT, SOLVER_AUTO_SMALL = 0, 1, 2
SOLVERS = {"auto": SOLVER_AUTO, "exact": SOLVER_EXACT, "auto_small": SOLVER_AUTO_SMALL}
LAUNCH_GRID, LAUNCH_PERSISTENT = 0, 1
LAUNCHES = {"grid": LAUNCH_GRID, "persistent": LAUNCH_PERSISTENT}
BC_PERIODIC, BC_TRANSMISSIVE = 0, 1
SCHEME_SEMI_IMPLICIT, SCHEME_EXPLICIT, SCHEME_SGN = 0, 1, 2


class HsgnParams(C.Structure):
    _fields_ = [("g", C.c_double), ("lam", C.c_double), ("dx", C.c_double), ("cfl", C.c_double),
                ("mcfl", C.c_double), ("dt_fixed", C.c_double), ("t_end", C.c_double),
                ("bc", C.c_int32), ("has_bathymetry", C.c_int32), ("order", C.c_int32),
                ("scheme", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhsgn.so is not built (run __graft_entry__.build()); "
                               "there is no CPU fallback")
        L = C.CDLL(LIB_PATH)
        vp, dp = C.c_void_p, C.c_void_p
        L.hsgn_init.restype = C.c_int
        L.hsgn_init.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(C.c_int64),
                                C.POINTER(HsgnParams), dp, vp]
        L.hsgn_set_state.restype = C.c_int
        L.hsgn_set_state.argtypes = [vp, dp, dp, dp, dp, dp]
        L.hsgn_get_state.restype = C.c_int
        L.hsgn_get_state.argtypes = [vp, dp, dp, dp, dp, dp]
        L.hsgn_get_dt.restype = C.c_int
        L.hsgn_get_dt.argtypes = [vp, dp]
        L.hsgn_step.restype = C.c_int
        L.hsgn_step.argtypes = [vp, C.c_int32]
        L.hsgn_run.restype = C.c_int
        L.hsgn_run.argtypes = [vp, C.c_int32, C.c_int32]
        L.hsgn_step_timed.restype = C.c_int
        L.hsgn_step_timed.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.hsgn_set_solver.restype = C.c_int
        L.hsgn_set_solver.argtypes = [vp, C.c_int32]
        L.hsgn_plan_info.restype = C.c_int
        L.hsgn_plan_info.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.hsgn_autotune.restype = C.c_int
        L.hsgn_autotune.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.hsgn_adjoint.restype = C.c_int
        L.hsgn_adjoint.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, vp, vp, vp, vp, vp, vp]
        L.hsgn_status.restype = C.c_int
        L.hsgn_status.argtypes = [vp, C.POINTER(C.c_int32)]
        L.hsgn_last_error.restype = C.c_char_p
        L.hsgn_last_error.argtypes = [vp]
        L.hsgn_version.restype = C.c_char_p
        L.hsgn_destroy.restype = None
        L.hsgn_destroy.argtypes = [vp]
        L.hsgn_set_instance_solvers.restype = C.c_int
        L.hsgn_set_instance_solvers.argtypes = [vp, C.POINTER(C.c_int32)]
        L.hsgn_autotune_classes.restype = C.c_int
        L.hsgn_autotune_classes.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                            C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                            C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                            C.POINTER(C.c_double)]
        L.hsgn_set_halo_margin.restype = C.c_int
        L.hsgn_set_halo_margin.argtypes = [vp, C.c_double]
        L.hsgn_set_launch.restype = C.c_int
        L.hsgn_set_launch.argtypes = [vp, C.c_int32]
        L.hsgn_set_adjoint_tape_bytes.restype = C.c_int
        L.hsgn_set_adjoint_tape_bytes.argtypes = [vp, C.c_int64]
        L.hsgn_set_halo_retry.restype = C.c_int
        L.hsgn_set_halo_retry.argtypes = [vp, C.c_int32]
        L.hsgn_halo_state.restype = C.c_int
        L.hsgn_halo_state.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.hsgn_autotune_launch.restype = C.c_int
        L.hsgn_autotune_launch.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.hsgn_step_noalloc.restype = C.c_int
        L.hsgn_step_noalloc.argtypes = [C.c_int32, C.POINTER(C.c_int64), C.POINTER(HsgnParams),
                                        dp, dp, dp, dp, dp, dp, C.c_int32, C.c_int32, vp,
                                        C.POINTER(C.c_int32), C.c_char_p]
        _lib = L
    return _lib


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


class HsgnError(RuntimeError):
    pass


class Solver:
    """A batch of independent hSGN instances on one GPU.

    offsets: int64 sequence (n_inst + 1); params: list of dicts with keys
    g, lam, dx, cfl, mcfl, dt_fixed, t_end, bc, has_b; b: float64 device
    tensor (sum of sizes) or None.
    """

    def __init__(self, offsets, params, b=None, device="cuda", stream=None):
        L = lib()
        self.device = torch.device(device)
        offs = np.ascontiguousarray(offsets, dtype=np.int64)
        self.n_inst = len(offs) - 1
        self.ncell = int(offs[-1])
        pa = _params_array(params)
        self._offsets = offs
        self._params = [dict(p) for p in params]
        if b is not None:
            b = b.to(self.device, torch.float64).contiguous()
        self._b = b
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._stream = s
        h = C.c_void_p()
        rc = L.hsgn_init(C.byref(h), self.n_inst, offs.ctypes.data_as(C.POINTER(C.c_int64)), pa,
                         _ptr(b), C.c_void_p(s.cuda_stream))
        if rc != HSGN_OK:
            raise HsgnError("hsgn_init failed (%d)" % rc)
        self._h = h

    def set_solver(self, mode):
        """mode: "auto" (windowed single pass where certified), "exact"
        (two-pass partition solve) or "auto_small" (2048-row windows, 256
        threads)."""
        m = SOLVERS[mode] if isinstance(mode, str) else int(mode)
        self._check(lib().hsgn_set_solver(self._h, m), "hsgn_set_solver")

    def autotune(self, nsteps=4):
        """Time every solver mode on the loaded state, keep the fastest, leave
        the state unchanged.  Returns (kept mode name, {mode name: ms/step})."""
        ms = (C.c_double * 3)()
        mode = C.c_int32(0)
        self._check(lib().hsgn_autotune(self._h, int(nsteps), ms, C.byref(mode)), "hsgn_autotune")
        names = {v: k for k, v in SOLVERS.items()}
        return names[mode.value], {names[m]: ms[m] for m in range(3)}

    def set_halo_margin(self, margin):
        """Safety factor of the windowed solves' halo estimates (default 2);
        re-plans at once."""
        self._check(lib().hsgn_set_halo_margin(self._h, float(margin)), "hsgn_set_halo_margin")

    def set_adjoint_tape_bytes(self, nbytes):
        """Tape budget of the adjoint in bytes: every segment is taped in the
        forward pass (nothing recomputed) when all tapes fit; 0 always
        recomputes; negative: half the free device memory (the default)."""
        self._check(lib().hsgn_set_adjoint_tape_bytes(self._h, int(nbytes)),
                    "hsgn_set_adjoint_tape_bytes")

    def set_halo_retry(self, enable=True):
        """Halo retry: a block whose windows could not certify their
        truncation is run again from a copy of its initial state, the
        flagged instances at twice their halo margin (hsgn_run and
        hsgn_step then synchronise)."""
        self._check(lib().hsgn_set_halo_retry(self._h, 1 if enable else 0), "hsgn_set_halo_retry")

    def halo_state(self):
        """(halo margin of every instance, blocks run again since the state
        was loaded)."""
        m = np.zeros(self.n_inst, dtype=np.float64)
        r = C.c_int32()
        self._check(lib().hsgn_halo_state(self._h, m.ctypes.data_as(C.POINTER(C.c_double)),
                                          C.byref(r)), "hsgn_halo_state")
        return m, r.value

    def set_launch(self, launch):
        """Window-stage launch: "grid" (one workgroup per window) or
        "persistent" (resident workgroups walking per-XCD work queues)."""
        k = LAUNCHES[launch] if isinstance(launch, str) else int(launch)
        self._check(lib().hsgn_set_launch(self._h, k), "hsgn_set_launch")

    def autotune_launch(self, nsteps=4):
        """Time both window-stage launches on the current plan, keep the
        faster, leave the state unchanged.  Returns (kept launch name,
        {launch name: ms/step})."""
        ms = (C.c_double * 2)()
        k = C.c_int32(0)
        self._check(lib().hsgn_autotune_launch(self._h, int(nsteps), ms, C.byref(k)),
                    "hsgn_autotune_launch")
        names = {v: n for n, v in LAUNCHES.items()}
        return names[k.value], {names[i]: ms[i] for i in range(2)}

    def set_instance_solvers(self, modes):
        """Per-instance solver modes (names or HSGN_SOLVER_* values)."""
        m = np.ascontiguousarray([SOLVERS[x] if isinstance(x, str) else int(x) for x in modes],
                                 dtype=np.int32)
        assert len(m) == self.n_inst
        self._check(lib().hsgn_set_instance_solvers(self._h, m.ctypes.data_as(C.POINTER(C.c_int32))),
                    "hsgn_set_instance_solvers")

    def autotune_classes(self, nsteps=4, max_classes=256):
        """hsgn_autotune_classes: the per-class autotuner table (a dict that
        json can store) and the plan it kept."""
        P32, PD = C.POINTER(C.c_int32), C.POINTER(C.c_double)
        ncls = C.c_int32(0)
        cls = np.zeros(self.n_inst, dtype=np.int32)
        keys = np.zeros((max_classes, 4), dtype=np.int32)
        ms = np.zeros((max_classes, 3), dtype=np.float64)
        kept = np.zeros(max_classes, dtype=np.int32)
        whole = np.zeros(5, dtype=np.float64)
        self._check(lib().hsgn_autotune_classes(self._h, int(nsteps), int(max_classes),
                                                C.byref(ncls), cls.ctypes.data_as(P32),
                                                keys.ctypes.data_as(P32), ms.ctypes.data_as(PD),
                                                kept.ctypes.data_as(P32), whole.ctypes.data_as(PD)),
                    "hsgn_autotune_classes")
        names = {v: k for k, v in SOLVERS.items()}
        sizes = np.diff(self._offsets)
        table = []
        for q in range(ncls.value):
            sel = cls == q
            table.append({"key": {"n_bucket": int(keys[q, 0]), "bc": int(keys[q, 1]),
                                  "bed": int(keys[q, 2]), "halo_bucket": int(keys[q, 3])},
                          "instances": int(sel.sum()), "cells": int(sizes[sel].sum()),
                          "ms_per_step": {names[m]: round(float(ms[q, m]), 4) for m in range(3)},
                          "kept": names[int(kept[q])]})
        kept_plan = "per_class" if whole[4] < 0 else names[int(whole[4])]
        return {"classes": table, "kept": kept_plan,
                "whole_batch_ms_per_step": {**{names[m]: round(float(whole[m]), 4) for m in range(3)},
                                            "per_class": round(float(whole[3]), 4)}}

    def apply_table(self, table):
        """The plan a stored table (autotune_classes) kept: a uniform mode, or
        per-instance modes where each instance takes the mode kept for its
        class key (instances whose key the table lacks take the table's most
        common mode)."""
        if table["kept"] != "per_class":
            self.set_solver(table["kept"])
            return
        keymode = {tuple(c["key"][k] for k in ("n_bucket", "bc", "bed", "halo_bucket")): c["kept"]
                   for c in table["classes"]}
        modes = [c["kept"] for c in table["classes"]]
        default = max(set(modes), key=modes.count) if modes else "auto"
        keys = self.class_keys()
        self.set_instance_solvers([keymode.get(tuple(k), default) for k in keys])

    def class_keys(self):
        """Class key (N bucket, bc, bed, halo bucket) of every instance, as the
        library's tuner forms it (the halo from the plan of the loaded state)."""
        info = self.plan_info()
        sizes = np.diff(self._offsets)
        out = []
        for j in range(self.n_inst):
            nb = 0
            while (1 << nb) < sizes[j]:
                nb += 1
            L = int(info["halo"][j])
            hb = 0
            while L > 0 and (1 << hb) < L and hb < 30:
                hb += 1
            out.append((nb, int(self._params[j]["bc"]), int(self._params[j]["has_b"]), hb))
        return out

    def plan_info(self):
        mode = np.zeros(self.n_inst, dtype=np.int32)
        halo = np.zeros(self.n_inst, dtype=np.int32)
        cnt = np.zeros(4, dtype=np.int32)
        P = C.POINTER(C.c_int32)
        self._check(lib().hsgn_plan_info(self._h, mode.ctypes.data_as(P), halo.ctypes.data_as(P),
                                         cnt.ctypes.data_as(P)), "hsgn_plan_info")
        return dict(mode=mode, halo=halo, windows=int(cnt[0]), exact_tiles=int(cnt[1]),
                    exact_multi=int(cnt[2]), window_rows=int(cnt[3]),
                    window_launches=(2 if int(cnt[3]) < 0 else (1 if int(cnt[0]) > 0 else 0)))

    @classmethod
    def from_workload(cls, wl, device="cuda", solver=None, order=2, scheme=SCHEME_SEMI_IMPLICIT,
                      cfl=None):
        """order 2: the two-stage IMEX step; 1: the first-order scheme.
        scheme SCHEME_EXPLICIT: the explicit Heun step (flat bottom); cfl, if
        given, replaces the workload's CFL number."""
        params = [dict(g=wl.g[j], lam=wl.lam[j], dx=wl.dx[j],
                       cfl=wl.cfl[j] if cfl is None else cfl, mcfl=wl.mcfl[j],
                       dt_fixed=wl.dt_fixed[j], t_end=wl.t_end[j], bc=wl.bc[j], has_b=wl.has_b[j],
                       order=order, scheme=scheme)
                  for j in range(wl.n_inst)]
        b = None if wl.b is None else torch.from_numpy(wl.b).to(device)
        s = cls(wl.offsets, params, b, device=device)
        s.set_state(*[torch.from_numpy(a).to(device) for a in wl.state()])
        if solver is not None:
            s.set_solver(solver)
        return s

    def _check(self, rc, what):
        if rc != HSGN_OK:
            msg = lib().hsgn_last_error(self._h).decode()
            raise HsgnError("%s failed (%d): %s" % (what, rc, msg))

    def set_state(self, h, q, m=None, W=None, t=None):
        self._keep = (h, q, m, W, t)
        self._check(lib().hsgn_set_state(self._h, _ptr(h), _ptr(q), _ptr(m), _ptr(W), _ptr(t)),
                    "hsgn_set_state")

    def get_state(self):
        out = [torch.empty(self.ncell, dtype=torch.float64, device=self.device) for _ in range(4)]
        t = torch.empty(self.n_inst, dtype=torch.float64, device=self.device)
        self._check(lib().hsgn_get_state(self._h, *[_ptr(a) for a in out], _ptr(t)), "hsgn_get_state")
        return tuple(out), t

    def get_dt(self):
        d = torch.empty(self.n_inst, dtype=torch.float64, device=self.device)
        self._check(lib().hsgn_get_dt(self._h, _ptr(d)), "hsgn_get_dt")
        return d

    def step(self, nsteps=1):
        self._check(lib().hsgn_step(self._h, int(nsteps)), "hsgn_step")

    def run(self, nsteps, block=100):
        self._check(lib().hsgn_run(self._h, int(nsteps), int(block)), "hsgn_run")

    def step_timed(self, nsteps=1):
        """Eager steps with HIP events around every launch; returns
        {kind: (total_ms, launches)}."""
        ms = (C.c_double * len(KERNEL_KINDS))()
        cnt = (C.c_int32 * len(KERNEL_KINDS))()
        self._check(lib().hsgn_step_timed(self._h, int(nsteps), ms, cnt), "hsgn_step_timed")
        return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNEL_KINDS)}

    def adjoint(self, nsteps, K, gauges, targets, zeta0, grad=True):
        """Gauge-misfit loss per instance and its gradients with respect to the
        initial free surface zeta0 and the bed (hand-written discrete adjoint,
        checkpoints every K steps).  gauges: int32 (n_inst, n_gauge) cells
        relative to their instance; targets: (n_inst, nsteps, n_gauge);
        zeta0: (ncell,).  Returns (loss, grad_zeta0, grad_b); with
        grad=False only the loss is computed and the gradients are None."""
        dev = self.device
        g = gauges.to(dev, torch.int32).contiguous()
        tg = targets.to(dev, torch.float64).contiguous()
        z = zeta0.to(dev, torch.float64).contiguous()
        assert g.shape[0] == self.n_inst and tg.shape == (self.n_inst, nsteps, g.shape[1])
        loss = torch.empty(self.n_inst, dtype=torch.float64, device=dev)
        gz = torch.empty(self.ncell, dtype=torch.float64, device=dev) if grad else None
        gb = torch.empty(self.ncell, dtype=torch.float64, device=dev) if grad else None
        self._keep_adj = (g, tg, z)
        self._check(lib().hsgn_adjoint(self._h, int(nsteps), int(K), int(g.shape[1]),
                                       C.c_void_p(g.data_ptr()), _ptr(tg), _ptr(z), _ptr(loss),
                                       _ptr(gz), _ptr(gb)), "hsgn_adjoint")
        return loss, gz, gb

    def status(self):
        f = np.zeros(self.n_inst, dtype=np.int32)
        rc = lib().hsgn_status(self._h, f.ctypes.data_as(C.POINTER(C.c_int32)))
        return rc, f

    def close(self):
        if getattr(self, "_h", None):
            lib().hsgn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


MSG_LEN = 512  # HSGN_MSG_LEN
NOALLOC_MAX_CELLS, NOALLOC_MAX_INST = 1 << 20, 4096


def _params_array(params):
    pa = (HsgnParams * len(params))()
    for j, p in enumerate(params):
        pa[j] = HsgnParams(p["g"], p["lam"], p["dx"], p["cfl"], p["mcfl"], p["dt_fixed"],
                           p["t_end"], int(p["bc"]), int(p["has_b"]), int(p.get("order", 2)),
                           int(p.get("scheme", SCHEME_SEMI_IMPLICIT)))
    return pa


def step_noalloc(offsets, params, b, h, q, m, W, t=None, nsteps=1, solver="auto", stream=None):
    """hsgn_step_noalloc: advance the state tensors (h, q, m, W; t if given)
    in place by nsteps semi-implicit steps without any device allocation by
    the library.  Returns (rc, flags, message)."""
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    n_inst = len(offs) - 1
    pa = _params_array(params)
    flags = np.zeros(n_inst, dtype=np.int32)
    msg = C.create_string_buffer(MSG_LEN)
    s = stream if stream is not None else torch.cuda.current_stream(h.device)
    m_ = SOLVERS[solver] if isinstance(solver, str) else int(solver)
    rc = lib().hsgn_step_noalloc(n_inst, offs.ctypes.data_as(C.POINTER(C.c_int64)), pa, _ptr(b),
                                 _ptr(h), _ptr(q), _ptr(m), _ptr(W), _ptr(t), int(nsteps), m_,
                                 C.c_void_p(s.cuda_stream),
                                 flags.ctypes.data_as(C.POINTER(C.c_int32)), msg)
    return rc, flags, msg.value.decode()


class HsgnAdjointFn(torch.autograd.Function):
    """loss = HsgnAdjointFn.apply(zeta0, b, spec): per-instance gauge misfit
    of a batch started from rest with free surface zeta0 over bed b (both
    float64 tensors on the GPU).  spec: dict with offsets, params (list of
    dicts, dt_fixed > 0), nsteps, K, gauges, targets.  The backward pass uses
    the gradients the hand-written adjoint computed with the loss."""

    @staticmethod
    def forward(ctx, zeta0, b, spec):
        s = Solver(spec["offsets"], spec["params"], b.detach(), device=zeta0.device)
        try:
            loss, gz, gb = s.adjoint(spec["nsteps"], spec["K"], spec["gauges"], spec["targets"],
                                     zeta0.detach())
        finally:
            s.close()
        offs = torch.as_tensor(np.asarray(spec["offsets"]), device=zeta0.device)
        inst_of_cell = torch.repeat_interleave(torch.arange(len(offs) - 1, device=zeta0.device),
                                               offs[1:] - offs[:-1])
        ctx.save_for_backward(gz, gb, inst_of_cell)
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        gz, gb, inst_of_cell = ctx.saved_tensors
        w = grad_loss[inst_of_cell]
        return w * gz, w * gb, None
