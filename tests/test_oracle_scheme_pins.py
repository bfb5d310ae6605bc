"""Pins of the oracle's semi-implicit stage that do not restate its formulas.

- Consistency with the bathymetric hSGN system (Sec. 2.3, eq. hSGNb_eq): as
  tau -> 0, (U_new - U)/tau of one stage must converge, at second order in
  dx, to the right-hand side of the PDE, written for m = h eta (the exact
  rewrite of the h eta-tilde equation since b_t = 0) and evaluated with
  spectral derivatives of trigonometric polynomials (exact to rounding).
  The first-order term in tau of the depth quotient is -d/dx of the
  momentum right-hand side (the mass flux uses the implicitly updated
  momentum, Sec. 3.1 eq. hSGN_eq-split-I); it pins the face force of the
  depth system, bed terms included, which the tau -> 0 limit cannot see.
- Linear stability at rest of one two-stage step (still water on a small
  periodic mesh; it is what fixes the Rusanov speed |u| + sqrt(g h) over
  the printed |u|): spectral radius of the step's Jacobian, by complex
  steps.
- Mode A, the printed lines of Sec. 4.2 (eq. GN_hyp_eq_semi_fully_discrete),
  against the P-form the oracle and the library use: same limit, difference
  O(dx^2) on the solitary wave at lambda = 100; mode A breaks down at
  lambda = 1e4 where the P-form runs.
- Self-convergence over a bed.
- Planted mistakes: each of these pins fails on the oracle built with a
  mistake it is meant to catch (a doubled p~ factor, a doubled bed source of
  h eta, the printed Rusanov speed |u|, a sign slip in the P-form).
"""
import os

import numpy as np
import pytest

import oracle as O
from paper_2510_07539_amd import workloads as WL

G = 9.81


# ---------------------------------------------------------------------------
# Consistency with eq. hSGNb_eq
# ---------------------------------------------------------------------------
LX = 10.0
KX = 2.0 * np.pi / LX


def _fields(x):
    """Smooth periodic depth, velocity, eta/h, w and bed (trigonometric
    polynomials, so every flux below is one too)."""
    h = 1.0 + 0.1 * np.sin(KX * x) + 0.03 * np.cos(2 * KX * x + 0.4)
    u = 0.3 * np.cos(KX * x + 0.7)
    r = 1.0 + 0.02 * np.sin(KX * x + 1.1)  # eta / h
    w = 0.05 * np.sin(2 * KX * x)
    b = 0.2 + 0.15 * np.cos(KX * x + 0.3)
    return h, u, r, w, b


def _ddx(f):
    """Spectral derivative on the periodic grid: exact to rounding for a
    trigonometric polynomial of degree below N/2."""
    n = len(f)
    k = 2.0 * np.pi * np.fft.fftfreq(n, d=LX / n)
    return np.real(np.fft.ifft(1j * k * np.fft.fft(f)))


def _pde_rhs(N, lam):
    """Point values at cell centres of the state and of the right-hand side
    of eq. hSGNb_eq with m = h eta:
      h_t = -(h u)_x
      q_t = -(h u^2 + g h^2/2 + eta p~)_x - (g h + (3/2) p~) b_x
      m_t = -(h u eta)_x + h w - (3/2) h u b_x
      W_t = -(h u w)_x + 3 p~,       p~ = (lambda/3)(1 - eta/h)."""
    dx = LX / N
    x = (np.arange(N) + 0.5) * dx
    h, u, r, w, b = _fields(x)
    eta = r * h
    pt = lam / 3.0 * (1.0 - r)
    Rh = -_ddx(h * u)
    Rq = -_ddx(h * u * u + 0.5 * G * h * h + eta * pt) - (G * h + 1.5 * pt) * _ddx(b)
    Rm = -_ddx(h * u * eta) + h * w - 1.5 * h * u * _ddx(b)
    RW = -_ddx(h * u * w) + 3.0 * pt
    U = (h, h * u, h * eta, h * w)
    return U, b, (Rh, Rq, Rm, RW), -_ddx(Rq)


def _stage_taylor(N, lam):
    """U_new(tau) of one stage from U_E = U_old = U at tau = +-s, +-2s
    (s = 1e-3 dx): Richardson-extrapolated first and second tau-derivatives
    at 0.  Returns (U, R, -d/dx R_q, dU/dtau, (1/2) d2U/dtau2)."""
    U, b, R, dRq = _pde_rhs(N, lam)
    dx = LX / N
    p = O.make_params(lam=lam, dx=dx, bc=O.BC_PERIODIC, has_b=1)

    def at(tau):
        rc, Un = O.stage(p, tau, b, U, U)
        assert rc == 0
        return np.array(Un)

    s = 1e-3 * dx
    U0 = np.array(U)
    Up, Um, Up2, Um2 = at(s), at(-s), at(2 * s), at(-2 * s)
    d1 = (4.0 * (Up - Um) / (2 * s) - (Up2 - Um2) / (4 * s)) / 3.0
    d2 = (4.0 * (Up - 2 * U0 + Um) / (2 * s * s) - (Up2 - 2 * U0 + Um2) / (8 * s * s)) / 3.0
    return U0, R, dRq, d1, d2


def consistency_errors(lam=50.0, Ns=(64, 128, 256)):
    """Max-norm errors per field of the tau -> 0 quotient against the PDE,
    and of the first-order tau term of the depth against -d/dx R_q."""
    e0, e1 = [], []
    for N in Ns:
        _, R, dRq, d1, d2 = _stage_taylor(N, lam)
        e0.append([np.max(np.abs(d1[f] - R[f])) for f in range(4)])
        e1.append(np.max(np.abs(d2[0] - dRq)))
    return np.array(e0), np.array(e1)


def _assert_second_order(e, what):
    e = np.asarray(e)
    assert np.all(e[:-1] / e[1:] > 3.6), (what, e)


@pytest.mark.parametrize("lam", [50.0, 1000.0])
def test_stage_consistent_with_bathymetric_hsgn(lam):
    e0, e1 = consistency_errors(lam)
    for f in range(4):
        _assert_second_order(e0[:, f], "hqmW"[f])
    # the finest errors are small against the right-hand sides (O(1))
    assert np.all(e0[-1] < [1e-4, 1e-3, 1e-4, 1e-4]), e0[-1]


@pytest.mark.parametrize("lam", [50.0, 1000.0])
def test_stage_face_force_consistent_with_momentum_balance(lam):
    e0, e1 = consistency_errors(lam)
    _assert_second_order(e1, "tau term of the depth")
    assert e1[-1] < 2e-3, e1


# ---------------------------------------------------------------------------
# Linear stability of the two-stage step at rest
# ---------------------------------------------------------------------------
def rest_spectral_radius(lam, N, dx, h0, bc, bed=False, cfl=0.9):
    """Spectral radius of one step's Jacobian at still water (u = 0,
    eta = h, w = 0) with the step's dt fixed at its CFL value; with a bed,
    the trapezoidal bar of the batched workload (toe at a quarter)."""
    x = (np.arange(N) + 0.5) * dx
    b = WL.trapezoid_bar(x, 0.25 * N * dx) if bed else None
    h = h0 - (b if bed else 0.0) * np.ones(N)
    U = (h, np.zeros(N), h * h, np.zeros(N))
    dt = cfl * dx / np.sqrt(G * h.max())
    p = O.make_params(lam=lam, dx=dx, bc=bc, has_b=int(bed), dt_fixed=dt)
    rc, J = O.step_jacobian(p, b, U)
    assert rc == 0
    return float(np.max(np.abs(np.linalg.eigvals(J))))


STABLE_CASES = [
    # (lam, N, dx, h0, bc, bed): still water on a small mesh (h0 = 1,
    # dx = 0.25), the bar of the batched and gradient workloads
    # (transmissive, dx = 0.04), and the long periodic mesh (h0 = 1, dx = 0.01)
    (1e2, 32, 0.25, 1.0, 0, False),
    (1e4, 32, 0.25, 1.0, 0, False),
    (1e2, 32, 0.25, 1.0, 1, False),
    (1e4, 32, 0.25, 1.0, 1, False),
    (1e2, 400, 0.04, 0.4, 1, True),
    (1e4, 400, 0.04, 0.4, 1, True),
    (1e4, 64, 0.01, 1.0, 0, False),
]


@pytest.mark.parametrize("case", STABLE_CASES)
def test_si_rest_state_is_linearly_stable(case):
    lam, N, dx, h0, bc, bed = case
    rho = rest_spectral_radius(lam, N, dx, h0, bc, bed)
    assert rho <= 1.0 + 1e-7, rho


def test_si_long_wave_growth_at_lambda_1e4_is_recorded():
    """A finding, kept as a test so that a change of the scheme shows up
    here: on a periodic flat mesh with h0 = 0.4, dx = 0.04 and lambda = 1e4,
    the longest waves (k h0 ~ 2) grow by about 1.07e-4 per step at CFL 0.9
    (mode A equally); at CFL 0.6 the step is stable.  The batched and
    gradient workloads are transmissive, where the bar geometry is stable
    at the same lambda and dx (above)."""
    r9 = rest_spectral_radius(1e4, 32, 0.04, 0.4, 0, cfl=0.9)
    r6 = rest_spectral_radius(1e4, 32, 0.04, 0.4, 0, cfl=0.6)
    assert 5e-5 < r9 - 1.0 < 2e-4, r9
    assert r6 <= 1.0 + 1e-7, r6


# ---------------------------------------------------------------------------
# Mode A (the printed Sec. 4.2 lines) against the P-form
# ---------------------------------------------------------------------------
def _solitary(N, lam, form, nsteps=100000, t_end=10.0):
    wl = WL.solitary(N=N, lam=lam, t_end=t_end)
    n, prm, b, U0 = wl.instance(0)
    p = O.make_params(**prm, form=form)
    rc, U, t = O.run(p, b, U0, 0.0, nsteps)
    return rc, U, t


def mode_a_vs_p(Ns=(400, 800, 1600), lam=100.0):
    """L1 (mean |.|) of A - P in the depth after the solitary wave's 10 s,
    and both L1 errors against the SGN closed form at N = 800."""
    dAP, errs = [], {}
    for N in Ns:
        rcA, UA, tA = _solitary(N, lam, O.FORM_A)
        rcP, UP, tP = _solitary(N, lam, O.FORM_P)
        assert rcA == 0 and rcP == 0 and tA == tP == 10.0
        dAP.append(np.mean(np.abs(UA[0] - UP[0])))
        if N == 800:
            x = (np.arange(N) + 0.5) * (200.0 / N)
            he, _, _ = WL.soliton(x, 1.0, 0.2, 100.0, t=10.0)
            errs = dict(A=np.mean(np.abs(UA[0] - he)), P=np.mean(np.abs(UP[0] - he)))
    return np.array(dAP), errs


def test_mode_a_agrees_with_p_form_to_second_order():
    """Solitary wave (N = 800 on [0, 200], lambda = 100, t = 10 s): both
    forms approximate the same equations, so A - P falls like dx^2
    (measured 7.4e-5, 1.75e-5, 4.2e-6); against the SGN closed form the
    L1 depth errors are 4.26e-4 (A) and 4.15e-4 (P)."""
    d, errs = mode_a_vs_p()
    _assert_second_order(d, "A - P")
    assert d[1] < 3e-5, d
    assert errs["A"] == pytest.approx(4.26e-4, rel=0.03), errs
    assert errs["P"] == pytest.approx(4.15e-4, rel=0.03), errs


def test_mode_a_breaks_down_at_lambda_1e4():
    """Where mode A fails: at lambda = 1e4 (N = 800, dx = 0.25) the printed
    scheme loses coercivity (beta <= 0) at step 30, while the P-form runs
    200 steps.  Its face terms cancel the O(lambda) pressure only up to
    O(lambda dx^2 / beta_1)."""
    wl = WL.solitary(N=800, lam=1e4, t_end=0.0)
    n, prm, b, U = wl.instance(0)
    pA = O.make_params(**prm, form=O.FORM_A)
    t = 0.0
    fail = None
    for s in range(200):
        rc, U, t, _ = O.step(pA, b, U, t)
        if rc:
            fail = (s + 1, rc)
            break
    assert fail is not None and 20 <= fail[0] <= 40, fail
    rcP, UP, _ = _solitary(800, 1e4, O.FORM_P, nsteps=200, t_end=0.0)
    assert rcP == 0 and np.all(np.isfinite(UP[0]))


def test_mode_a_rejects_a_bed():
    wl = WL.lake_at_rest(N=64)
    n, prm, b, U = wl.instance(0)
    rc, _, _, _ = O.step(O.make_params(**prm, form=O.FORM_A), b, U, 0.0)
    assert rc == O.EINVAL


# ---------------------------------------------------------------------------
# Self-convergence over a bed
# ---------------------------------------------------------------------------
def test_second_order_self_convergence_over_a_bed():
    """Solitary wave (a = 0.2 on a 1 m free surface) travelling over the
    smooth periodic bed b = 0.1 (1 + cos(2 pi x / 200)) for 3 s, lambda =
    100: successive differences of the depth (restricted to the coarsest
    mesh by cell averages) fall by about 4 per refinement."""
    sols = []
    for N in (400, 800, 1600, 3200):
        L = 200.0
        dx = L / N
        x = (np.arange(N) + 0.5) * dx
        b = 0.1 * (1.0 + np.cos(2 * np.pi * x / L))
        hs, u, ux = WL.soliton(x, 1.0, 0.2, 0.5 * L)
        h = hs - b
        part = WL._part(N, dx, 100.0, WL.BC_PERIODIC, h, u, ux, b=b, cfl=0.45, t_end=3.0)
        wl = WL._pack("bed convergence", [part], 100000)
        n, prm, bb, U = wl.instance(0)
        rc, Un, t = O.run(O.make_params(**prm), bb, U, 0.0, 100000)
        assert rc == 0 and t == 3.0
        sols.append(Un[0])

    def restrict(a, f):
        return a.reshape(-1, f).mean(1)

    d1 = np.abs(restrict(sols[1], 2) - sols[0]).sum()
    d2 = np.abs(restrict(sols[2], 4) - restrict(sols[1], 2)).sum()
    d3 = np.abs(restrict(sols[3], 8) - restrict(sols[2], 4)).sum()
    r1, r2 = d1 / d2, d2 / d3
    assert r1 > 3.3 and r2 > 3.5, (r1, r2)


# ---------------------------------------------------------------------------
# Planted mistakes: the pins above must catch each of them
# ---------------------------------------------------------------------------
MUTANTS = {
    # the p~ factor of the face force in the depth system doubled
    "face_force_pt_doubled": [
        ("gL[k] = (-beta[L] + db * (0.5 * g + 0.75 * phi[L])) / dx;",
         "gL[k] = (-beta[L] + db * (0.5 * g + 1.5 * phi[L])) / dx;"),
        ("gR[k] = (beta[R] + db * (0.5 * g + 0.75 * phi[R])) / dx;",
         "gR[k] = (beta[R] + db * (0.5 * g + 1.5 * phi[R])) / dx;"),
        ("g0[k] = (S[R] - S[L] + 0.75 * db * (T[L] + T[R])) / dx;",
         "g0[k] = (S[R] - S[L] + 1.5 * db * (T[L] + T[R])) / dx;"),
    ],
    # the p~ factor of the cell bed force in the momentum update doubled
    "cell_pt_doubled": [("0.5 * g * (hb[ip] + hb[im]) * dbc + 1.5 * pti * dbc);",
                         "0.5 * g * (hb[ip] + hb[im]) * dbc + 3.0 * pti * dbc);")],
    # the bed source -(3/2) q b_x of the h eta equation doubled
    "m_bed_source_doubled": [("- tau * 1.5 * qE[i] * dbc +", "- tau * 3.0 * qE[i] * dbc +")],
    # the gravity bed force taken from one side (first order in dx)
    "gravity_bed_one_sided": [("0.5 * g * (hb[ip] + hb[im]) * dbc", "g * hb[ip] * dbc")],
    # the printed Rusanov speed |u| of Sec. 4.1
    "speed_abs_u": [("if (!(RE(hL) > 0.0) || !(RE(hR) > 0.0)) rc = OR_ENONPHYS;\n"
                     "    real_t uL = qL / hL, uR = qR / hR;\n"
                     "    real_t sL = RABS(uL) + RSQRT(g * hL), sR = RABS(uR) + RSQRT(g * hR);",
                     "if (!(RE(hL) > 0.0) || !(RE(hR) > 0.0)) rc = OR_ENONPHYS;\n"
                     "    real_t uL = qL / hL, uR = qR / hR;\n"
                     "    real_t sL = RABS(uL), sR = RABS(uR);")],
    # sign slip in the P-form's S = P0 - beta h_E
    "pform_sign_slip": [("S[i] = P0[i] - beta[i] * h;", "S[i] = P0[i] + beta[i] * h;")],
}


def _consistency_pin():
    e0, e1 = consistency_errors(50.0)
    for f in range(4):
        _assert_second_order(e0[:, f], "hqmW"[f])
    assert np.all(e0[-1] < [1e-4, 1e-3, 1e-4, 1e-4]), e0[-1]


def _face_force_pin():
    e0, e1 = consistency_errors(50.0)
    _assert_second_order(e1, "tau term of the depth")
    assert e1[-1] < 2e-3, e1


def _stability_pin():
    for lam in (1e2, 1e4):
        rho = rest_spectral_radius(lam, 32, 0.25, 1.0, 0)
        assert rho <= 1.0 + 1e-7, rho


def _mode_a_pin():
    d, errs = mode_a_vs_p(Ns=(400, 800))
    _assert_second_order(d, "A - P")
    assert d[1] < 3e-5, d


CATCHES = {
    "face_force_pt_doubled": _face_force_pin,
    "cell_pt_doubled": _consistency_pin,
    "m_bed_source_doubled": _consistency_pin,
    "gravity_bed_one_sided": _consistency_pin,
    "speed_abs_u": _stability_pin,
    "pform_sign_slip": _mode_a_pin,
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    src = O.source_text()
    for old, new in MUTANTS[name]:
        assert src.count(old) == 1, (name, old)
        src = src.replace(old, new)
    O.build_at(str(tmp_path), src)
    pin = CATCHES[name]
    pin()  # passes on the oracle as built
    with O.using(str(tmp_path)):
        with pytest.raises(AssertionError):
            pin()
