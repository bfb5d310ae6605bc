"""Seeded synthetic workloads for the hSGN solver (inputs only).

This module holds the initial data of the test problems and nothing of the
numerical method: closed-form initial states, beds and the seeded random
draws.  Both the HIP library's tests/benchmark and the CPU oracle read the
same arrays produced here.

Initial data follow the solitary-wave test of Sec. 6.3 (closed form of the SGN
solitary wave; eta = h and w = -h u_x at t = 0), so m = h*eta = h^2 and
W = h*w = -h^2 u_x, sampled at cell centres.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

G = 9.81
BC_PERIODIC, BC_TRANSMISSIVE = 0, 1


@dataclass
class Workload:
    name: str
    offsets: np.ndarray            # int64, n_inst + 1
    g: np.ndarray                  # per-instance parameters (float64)
    lam: np.ndarray
    dx: np.ndarray
    cfl: np.ndarray
    mcfl: np.ndarray
    dt_fixed: np.ndarray
    t_end: np.ndarray
    bc: np.ndarray                 # int32
    has_b: np.ndarray              # int32
    b: np.ndarray | None           # bed, concatenated (None: flat everywhere)
    h: np.ndarray
    q: np.ndarray
    m: np.ndarray
    W: np.ndarray
    nsteps: int
    info: dict = field(default_factory=dict)

    @property
    def n_inst(self) -> int:
        return len(self.offsets) - 1

    @property
    def n_cells(self) -> int:
        return int(self.offsets[-1])

    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets)

    def state(self):
        return (self.h, self.q, self.m, self.W)

    def instance(self, j: int):
        """Slice of instance j: (n, params dict, b, (h, q, m, W))."""
        o0, o1 = int(self.offsets[j]), int(self.offsets[j + 1])
        prm = dict(g=float(self.g[j]), lam=float(self.lam[j]), dx=float(self.dx[j]),
                   cfl=float(self.cfl[j]), mcfl=float(self.mcfl[j]),
                   dt_fixed=float(self.dt_fixed[j]), t_end=float(self.t_end[j]),
                   bc=int(self.bc[j]), has_b=int(self.has_b[j]))
        b = None if (self.b is None or not self.has_b[j]) else self.b[o0:o1].copy()
        U = tuple(a[o0:o1].copy() for a in self.state())
        return o1 - o0, prm, b, U

    def subset(self, idx, name=None) -> "Workload":
        """A new workload made of the instances in idx (same data)."""
        idx = list(idx)
        sizes = self.sizes()[idx]
        offs = np.zeros(len(idx) + 1, dtype=np.int64)
        offs[1:] = np.cumsum(sizes)
        cat = lambda a: np.concatenate([a[int(self.offsets[j]):int(self.offsets[j + 1])] for j in idx])
        per = lambda a: np.ascontiguousarray(a[idx])
        return Workload(name or (self.name + "-subset"), offs, per(self.g), per(self.lam),
                        per(self.dx), per(self.cfl), per(self.mcfl), per(self.dt_fixed),
                        per(self.t_end), per(self.bc), per(self.has_b),
                        None if self.b is None else cat(self.b),
                        cat(self.h), cat(self.q), cat(self.m), cat(self.W), self.nsteps,
                        dict(self.info))


def _pack(name, parts, nsteps, info=None) -> Workload:
    """parts: list of dicts with keys n, g, lam, dx, cfl, mcfl, dt_fixed, t_end,
    bc, b (array or None), h, q, m, W."""
    sizes = np.array([p["n"] for p in parts], dtype=np.int64)
    offs = np.zeros(len(parts) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(sizes)
    f = lambda k: np.array([p[k] for p in parts], dtype=np.float64)
    any_b = any(p.get("b") is not None for p in parts)
    b = None
    if any_b:
        b = np.concatenate([p["b"] if p.get("b") is not None else np.zeros(p["n"]) for p in parts])
    has_b = np.array([1 if p.get("b") is not None else 0 for p in parts], dtype=np.int32)
    cat = lambda k: np.ascontiguousarray(np.concatenate([p[k] for p in parts]), dtype=np.float64)
    return Workload(name, offs, f("g"), f("lam"), f("dx"), f("cfl"), f("mcfl"), f("dt_fixed"),
                    f("t_end"), np.array([p["bc"] for p in parts], dtype=np.int32), has_b, b,
                    cat("h"), cat("q"), cat("m"), cat("W"), int(nsteps), info or {})


# --------------------------------------------------------------------------
# Closed forms
# --------------------------------------------------------------------------
def soliton(x, h0, a, x0, t=0.0, g=G):
    """SGN solitary wave (Sec. 6.3): h = h0 (1 + eps sech^2(kappa (x - x0 - C t))),
    u = C (1 - h0/h), C = sqrt(g h0 (1 + eps)), kappa = sqrt(3 eps / (4 h0^2 (1 + eps))).
    Returns (h, u, u_x) with u_x analytic."""
    eps = a / h0
    C = np.sqrt(g * h0 * (1.0 + eps))
    kap = np.sqrt(3.0 * eps / (4.0 * h0 * h0 * (1.0 + eps)))
    xi = np.clip(kap * (x - x0 - C * t), -300.0, 300.0)
    sech2 = 1.0 / np.cosh(xi) ** 2
    h = h0 * (1.0 + eps * sech2)
    u = C * (1.0 - h0 / h)
    hx = -2.0 * h0 * eps * kap * sech2 * np.tanh(xi)
    ux = C * h0 * hx / (h * h)
    return h, u, ux


def soliton_speed(h0, a, g=G):
    return float(np.sqrt(g * (h0 + a)))


def trapezoid_bar(x, toe, height=0.3, up=1.0 / 20.0, crest=2.0, down=1.0 / 10.0):
    """Submerged trapezoidal bar: rises from 0 at `toe` with slope `up` to
    `height`, flat crest of length `crest`, falls with slope `down`."""
    l_up = height / up
    l_dn = height / down
    x1, x2, x3 = toe + l_up, toe + l_up + crest, toe + l_up + crest + l_dn
    b = np.zeros_like(x)
    b = np.where((x >= toe) & (x < x1), (x - toe) * up, b)
    b = np.where((x >= x1) & (x < x2), height, b)
    b = np.where((x >= x2) & (x < x3), height - (x - x2) * down, b)
    return b


def _part(n, dx, lam, bc, h, u, ux, b=None, cfl=0.9, mcfl=0.5, t_end=0.0, dt_fixed=0.0, g=G):
    q = h * u
    return dict(n=int(n), g=g, lam=float(lam), dx=float(dx), cfl=cfl, mcfl=mcfl,
                dt_fixed=dt_fixed, t_end=t_end, bc=bc, b=b, h=np.ascontiguousarray(h),
                q=np.ascontiguousarray(q), m=np.ascontiguousarray(h * h),
                W=np.ascontiguousarray(-h * h * ux))


# --------------------------------------------------------------------------
# The five workloads (sizes as specified; unspecified details are stated)
# --------------------------------------------------------------------------
def solitary(N=800, L=200.0, h0=1.0, a=0.2, lam=100.0, x0=None, t_end=10.0, nsteps=None,
             bc=BC_PERIODIC) -> Workload:
    """C1: one solitary wave on a flat periodic bed, crest at the domain centre."""
    dx = L / N
    x = (np.arange(N) + 0.5) * dx
    x0 = 0.5 * L if x0 is None else x0
    h, u, ux = soliton(x, h0, a, x0)
    ns = nsteps if nsteps is not None else 100000
    return _pack("solitary", [_part(N, dx, lam, bc, h, u, ux, t_end=t_end)], ns,
                 dict(h0=h0, a=a, x0=x0, L=L))


def dam_break(N=20000, xa=-300.0, xb=300.0, hl=1.8, hr=1.0, width=0.3, lam=1000.0,
              nsteps=2000) -> Workload:
    """C2: dispersive dam break, transmissive.  The jump is smoothed with a
    tanh of half-width `width` (the paper smooths its bores the same way)."""
    dx = (xb - xa) / N
    x = xa + (np.arange(N) + 0.5) * dx
    h = 0.5 * (hl + hr) - 0.5 * (hl - hr) * np.tanh(x / width)
    z = np.zeros(N)
    return _pack("dam_break", [_part(N, dx, lam, BC_TRANSMISSIVE, h, z, z)], nsteps,
                 dict(width=width))


def batched_bar(n_inst=4096, seed=3, n_lo=512, n_hi=16384, dx=0.04, h0=0.4,
                lams=(100.0, 1000.0, 10000.0), nsteps=100) -> Workload:
    """C3: independent solitary waves over a submerged trapezoidal bar.
    Draw order from numpy's PCG64 default_rng(seed): N_j, a_j/h0, toe_j/L_j, lambda_j."""
    rng = np.random.default_rng(seed)
    Ns = rng.integers(n_lo, n_hi + 1, size=n_inst)
    amps = rng.uniform(0.05, 0.4, size=n_inst) * h0
    toes = rng.uniform(0.35, 0.45, size=n_inst)
    lam_j = rng.choice(np.asarray(lams, dtype=np.float64), size=n_inst)
    parts = []
    for j in range(n_inst):
        N = int(Ns[j])
        L = N * dx
        x = (np.arange(N) + 0.5) * dx
        b = trapezoid_bar(x, toes[j] * L)
        hs, u, ux = soliton(x, h0, amps[j], 0.2 * L)
        h = hs - b  # free surface zeta = h0 + soliton excess; depth = zeta - b
        parts.append(_part(N, dx, lam_j[j], BC_TRANSMISSIVE, h, u, ux, b=b))
    return _pack("batched_bar", parts, nsteps, dict(seed=seed))


def batched_flat(n_inst=4096, seed=3, n_lo=512, n_hi=16384, dx=0.04, h0=0.4,
                 lams=(100.0, 1000.0, 10000.0), nsteps=100) -> Workload:
    """Flat-bottom twin of the batched bar workload (the explicit scheme has
    no bed): the same draws from default_rng(seed) in the same order (the bar
    toe is drawn and unused), solitary waves on depth h0, transmissive."""
    rng = np.random.default_rng(seed)
    Ns = rng.integers(n_lo, n_hi + 1, size=n_inst)
    amps = rng.uniform(0.05, 0.4, size=n_inst) * h0
    rng.uniform(0.35, 0.45, size=n_inst)
    lam_j = rng.choice(np.asarray(lams, dtype=np.float64), size=n_inst)
    parts = []
    for j in range(n_inst):
        N = int(Ns[j])
        x = (np.arange(N) + 0.5) * dx
        h, u, ux = soliton(x, h0, amps[j], 0.2 * N * dx)
        parts.append(_part(N, dx, lam_j[j], BC_TRANSMISSIVE, h, u, ux))
    return _pack("batched_flat", parts, nsteps, dict(seed=seed))


def long_periodic(N=1 << 24, dx=0.01, lam=1e4, seed=4, K=16, nsteps=200) -> Workload:
    """C4: one long periodic mesh, h = 1 + sum_k a_k cos(2 pi k x / L + phi_k),
    a_k ~ U[0, 0.01], phi_k ~ U[0, 2 pi) drawn in that order from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    ak = rng.uniform(0.0, 0.01, size=K)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=K)
    L = N * dx
    x = (np.arange(N) + 0.5) * dx
    h = np.ones(N)
    for k in range(K):
        h += ak[k] * np.cos(2.0 * np.pi * (k + 1) * x / L + ph[k])
    z = np.zeros(N)
    return _pack("long_periodic", [_part(N, dx, lam, BC_PERIODIC, h, z, z)], nsteps,
                 dict(seed=seed))


def lake_at_rest(N=256, dx=0.04, h0=0.4, lam=100.0, bed=True, nsteps=100) -> Workload:
    """Still water over the bar (or flat): zeta = h0, u = 0."""
    x = (np.arange(N) + 0.5) * dx
    b = trapezoid_bar(x, 0.3 * N * dx) if bed else None
    h = h0 - (b if b is not None else 0.0)
    z = np.zeros(N)
    return _pack("lake_at_rest", [_part(N, dx, lam, BC_TRANSMISSIVE, h, z, z, b=b)], nsteps)


def concat(name, wls, nsteps=None) -> Workload:
    """Concatenate workloads into one batch."""
    parts = []
    for w in wls:
        for j in range(w.n_inst):
            n, prm, b, U = w.instance(j)
            d = dict(n=n, **{k: prm[k] for k in ("g", "lam", "dx", "cfl", "mcfl", "dt_fixed", "t_end", "bc")})
            d.update(b=b, h=U[0], q=U[1], m=U[2], W=U[3])
            parts.append(d)
    return _pack(name, parts, nsteps if nsteps is not None else wls[0].nsteps)


@dataclass
class AdjointCase:
    """Inputs of the gradient workload: a batch released from rest over a
    bar-plus-sinusoid bed, gauges, and the perturbed surface that defines the
    targets (the targets themselves come from running the forward solver)."""
    wl: Workload           # instances (params with dt_fixed) and bed; state = base surface at rest
    zeta0: np.ndarray      # base free surface
    zeta_target: np.ndarray  # perturbed free surface the targets are generated from
    gauges: np.ndarray     # int32 (n_inst, n_gauge), instance-relative cells
    nsteps: int
    K: int


def adjoint_bar(n_inst=1024, N=4096, dx=0.04, h0=0.4, lam=1000.0, seed=5, seed_target=55,
                nsteps=200, K=20, n_gauge=8, cfl=0.9, g=G) -> AdjointCase:
    """Gradient workload: bed b = trapezoidal bar (toe ~ U[0.4, 0.5] L) +
    0.02 sin(2 pi k_s x / L + phi_s), k_s ~ U{2..8}, phi_s ~ U[0, 2 pi)
    (default_rng(seed), drawn in that order per instance); base surface
    zeta0 = h0 + 0.05 exp(-(x - 0.2 L)^2 / 4) released from rest; targets from
    zeta0 + sum_{k=1..8} c_k sin(2 pi k x / L + psi_k), c_k ~ U[0, 2e-3],
    psi_k ~ U[0, 2 pi) (default_rng(seed_target)); gauges at cells
    floor((g + 1/2) N / n_gauge); fixed dt = cfl dx / max sqrt(g h) of the base
    state; transmissive."""
    rng = np.random.default_rng(seed)
    rng_t = np.random.default_rng(seed_target)
    L = N * dx
    x = (np.arange(N) + 0.5) * dx
    parts, zs, zts = [], [], []
    for j in range(n_inst):
        toe = rng.uniform(0.4, 0.5) * L
        ks = int(rng.integers(2, 9))
        ph = rng.uniform(0.0, 2.0 * np.pi)
        b = trapezoid_bar(x, toe) + 0.02 * np.sin(2.0 * np.pi * ks * x / L + ph)
        z = h0 + 0.05 * np.exp(-((x - 0.2 * L) ** 2) / 4.0)
        ck = rng_t.uniform(0.0, 2e-3, size=8)
        psi = rng_t.uniform(0.0, 2.0 * np.pi, size=8)
        zt = z.copy()
        for k in range(8):
            zt += ck[k] * np.sin(2.0 * np.pi * (k + 1) * x / L + psi[k])
        h = z - b
        dt = cfl * dx / np.sqrt(g * h.max())
        zero = np.zeros(N)
        parts.append(_part(N, dx, lam, BC_TRANSMISSIVE, h, zero, zero, b=b, dt_fixed=dt, g=g))
        zs.append(z)
        zts.append(zt)
    wl = _pack("adjoint_bar", parts, nsteps, dict(seed=seed))
    gauges = np.array([[int((gi + 0.5) * N / n_gauge) for gi in range(n_gauge)]] * n_inst,
                      dtype=np.int32)
    return AdjointCase(wl, np.concatenate(zs), np.concatenate(zts), gauges, nsteps, K)


# --------------------------------------------------------------------------
# The paper's other test problems (Sec. 6.1, 6.2, 6.4, 7) as seeded-free
# synthetic inputs.  Their reference solutions are not available; the
# library is checked against the oracle on them.  The paper runs them at
# larger CFL numbers with a Rusanov speed of |u|; with the speed
# |u| + sqrt(g h) used here they run at CFL 0.9.
# --------------------------------------------------------------------------
def gaussian_bell(N=5000, xa=-200.0, xb=200.0, A=1.0, h_inf=1.0, lam=100.0, nsteps=100,
                  bc=BC_TRANSMISSIVE) -> Workload:
    """Sec. 6.1: h = h_inf + A exp(-x^2 / 20) at rest over a flat bed."""
    dx = (xb - xa) / N
    x = xa + (np.arange(N) + 0.5) * dx
    h = h_inf + A * np.exp(-x * x / 20.0)
    z = np.zeros(N)
    return _pack("gaussian_bell", [_part(N, dx, lam, bc, h, z, z)], nsteps, dict(lam=lam))


def smooth_hump(N=5000, xa=-150.0, xb=150.0, A=1.0, h0=1.0, u0=1e-2, lam=500.0,
                nsteps=100) -> Workload:
    """Sec. 6.2: b = (h0 + A exp(-2 (x + 50)^2)) / 20, free surface
    h0 + A exp(-x^2), uniform velocity u0, transmissive."""
    dx = (xb - xa) / N
    x = xa + (np.arange(N) + 0.5) * dx
    b = (h0 + A * np.exp(-2.0 * (x + 50.0) ** 2)) / 20.0
    h = h0 + A * np.exp(-x * x) - b
    u = np.full(N, u0)
    z = np.zeros(N)
    return _pack("smooth_hump", [_part(N, dx, lam, BC_TRANSMISSIVE, h, u, z, b=b)], nsteps,
                 dict(lam=lam))


def favre(eps=1.1, N=5000, xa=-50.0, xb=50.0, h0=0.2, lam=100.0, nsteps=100, g=G) -> Workload:
    """Sec. 6.4: undular bore.  Upstream depth h1 = eps h0, jump velocity
    from the Rankine-Hugoniot condition, tanh transition of width 5 h0:
    h = h0 + (h1 - h0) s / 2, u = u1 s / 2, s = 1 - tanh(x / (5 h0))."""
    dx = (xb - xa) / N
    x = xa + (np.arange(N) + 0.5) * dx
    h1 = eps * h0
    u1 = np.sqrt(g * (h1 + h0) / (2.0 * h0 * h1)) * (h1 - h0)
    al = 5.0 * h0
    s = 1.0 - np.tanh(x / al)
    ds = -(1.0 - np.tanh(x / al) ** 2) / al
    h = h0 + 0.5 * (h1 - h0) * s
    u = 0.5 * u1 * s
    ux = 0.5 * u1 * ds
    return _pack("favre", [_part(N, dx, lam, BC_TRANSMISSIVE, h, u, ux, g=g)], nsteps,
                 dict(eps=eps, lam=lam))


def shelf(N=5000, L=280.0, h0=1.0, A=0.2, x0=80.0, lam=500.0, nsteps=100) -> Workload:
    """Sec. 7: solitary wave (crest at x0) travelling onto a 1:20 ramp from
    depth h0 to h0 - 0.5 between x = 130 and 140 m; transmissive."""
    dx = L / N
    x = (np.arange(N) + 0.5) * dx
    b = np.clip((x - 130.0) / 20.0, 0.0, 0.5)
    hs, u, ux = soliton(x, h0, A, x0)
    h = hs - b
    return _pack("shelf", [_part(N, dx, lam, BC_TRANSMISSIVE, h, u, ux, b=b)], nsteps,
                 dict(lam=lam))


def paper_tests(nsteps=100) -> Workload:
    """One batch of the four test problems above, at several lambda and bore
    amplitudes."""
    parts = [gaussian_bell(lam=100.0), gaussian_bell(lam=5000.0), smooth_hump(lam=500.0),
             favre(eps=1.1, lam=100.0), favre(eps=1.3, lam=500.0), shelf(lam=500.0)]
    return concat("paper_tests", parts, nsteps=nsteps)
