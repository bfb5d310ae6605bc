"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every test here checks the oracle (oracle/) against something other than
itself: closed forms, the un-eliminated linear system solved by dense LU,
the original implicit equations before elimination, finite-difference
derivatives of the paper's pressure law, conservation, lake at rest, the
SGN solitary wave, self-convergence, and the linear dispersion relation of
the hSGN system.  No GPU is used.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2510_07539_amd import workloads as WL

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rand_state(n, seed, amp=0.1, bed=False, h0=1.0):
    rng = np.random.default_rng(seed)
    x = np.linspace(0, 2 * np.pi, n, endpoint=False)
    h = h0 + amp * np.sin(x) + 0.05 * amp * rng.standard_normal(n)
    q = 0.3 * amp * np.cos(2 * x) + 0.05 * amp * rng.standard_normal(n)
    m = h * h * (1 + 0.01 * rng.standard_normal(n))
    W = 0.05 * rng.standard_normal(n)
    b = 0.1 * (1 + np.cos(x)) * h0 if bed else None
    return (h, q, m, W), b


# ---------------------------------------------------------------------------
# Tableau (Sec. 3.2, eq. tableau): golden fixture = the paper's printed table
# ---------------------------------------------------------------------------
def test_tableau_order_conditions_and_oracle_constants():
    with open(os.path.join(GOLD, "tableau.json")) as f:
        tab = json.load(f)
    gam = eval(tab["gamma"], {"sqrt": math.sqrt})
    c = eval(tab["c"], {"sqrt": math.sqrt, "gamma": gam})
    sub = {"gamma": gam, "c": c}
    AE = np.array([[eval(str(e), sub) for e in row] for row in tab["A_explicit"]])
    AI = np.array([[eval(str(e), sub) for e in row] for row in tab["A_implicit"]])
    bE = np.array([eval(str(e), sub) for e in tab["b_explicit"]])
    bI = np.array([eval(str(e), sub) for e in tab["b_implicit"]])
    cE, cI = AE.sum(1), AI.sum(1)
    # second order, including the coupling conditions of partitioned RK
    for bb in (bE, bI):
        assert abs(bb.sum() - 1) < 1e-15
    for bb in (bE, bI):
        for cc in (cE, cI):
            assert abs(bb @ cc - 0.5) < 1e-15
    # stiffly accurate implicit part: last row equals b, so R(inf) = 0
    assert np.allclose(AI[-1], bI, atol=0)
    Rinf = 1 - bI @ np.linalg.solve(AI, np.ones(2))
    assert abs(Rinf) < 1e-15
    # oracle literals are the efficient-form coefficients of this tableau
    g_o, e0, e1, t0, t1 = O.tableau()
    assert abs(g_o - gam) <= 1e-16
    assert abs(e1 - c / gam) < 4e-15 and abs(e0 - (1 - c / gam)) < 4e-15
    assert abs(t1 - (1 - gam) / gam) < 4e-15 and abs(t0 - (1 - (1 - gam) / gam)) < 4e-15
    # stage-2 combination reproduces the tableau rows: U_E^(2) = U^n + dt c H1
    # with dt H1 = (U_I^(1) - U^n)/gamma
    assert abs(e1 - c / gam) < 4e-15 and abs(t1 - AI[1, 0] / gam) < 4e-15


# ---------------------------------------------------------------------------
# Tridiagonal solver vs dense LU (plain and cyclic)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("cyclic", [False, True])
def test_tridiag_vs_dense(cyclic):
    rng = np.random.default_rng(7)
    for n in range(1, 33):
        lo = -rng.uniform(0.1, 1, n)
        up = -rng.uniform(0.1, 1, n)
        di = np.abs(lo) + np.abs(up) + rng.uniform(0.1, 2, n)
        rhs = rng.standard_normal(n)
        A = np.zeros((n, n))
        for i in range(n):
            A[i, i] += di[i]
            if i > 0:
                A[i, i - 1] += lo[i]
            elif cyclic:
                A[i, n - 1] += lo[i]
            if i < n - 1:
                A[i, i + 1] += up[i]
            elif cyclic:
                A[i, 0] += up[i]
        if not cyclic:
            lo[0] = 0.0
            up[-1] = 0.0
        rc, x = O.tridiag(lo, di, up, rhs, cyclic=cyclic)
        assert rc == 0
        xr = np.linalg.solve(A, rhs)
        assert np.max(np.abs(x - xr)) <= 1e-14 * max(1.0, np.max(np.abs(xr)))


# ---------------------------------------------------------------------------
# One stage: the un-eliminated coupled system (hbar, face momenta Q) solved by
# dense LU must give the oracle's hbar (Sec. 3.1 eq. hSGN_eq-split-I in the
# fully discrete form of Sec. 4.2).
# ---------------------------------------------------------------------------
def _uneliminated_hbar(n, p, tau, b, hE, ho, d):
    bc = p.bc
    dx, g = p.dx, p.g
    bb = np.zeros(n) if b is None else b
    nf = n if bc == 0 else n + 1

    def L_R(k):
        if bc == 0:
            return (k - 1) % n, k % n
        return max(k - 1, 0), min(k, n - 1)

    def residual(x):
        hb, Q = x[:n], x[n:]
        P = d["P0"] + d["beta"] * (hb - hE)
        pt = d["pt0"] + d["phi"] * (hb - hE)
        r = np.empty(n + nf)
        for k in range(nf):
            Lc, Rc = L_R(k)
            if bc != 0 and (k == 0 or k == n):
                r[n + k] = Q[k] - d["qd"][0 if k == 0 else n - 1]
                continue
            db = bb[Rc] - bb[Lc]
            G = (P[Rc] - P[Lc] + 0.5 * g * (hb[Lc] + hb[Rc]) * db
                 + 0.75 * (pt[Lc] + pt[Rc]) * db) / dx
            r[n + k] = Q[k] + tau * G - 0.5 * (d["qd"][Lc] + d["qd"][Rc])
        for i in range(n):
            Qr = Q[(i + 1) % nf] if bc == 0 else Q[i + 1]
            r[i] = hb[i] + tau / dx * (Qr - Q[i]) - ho[i]
        return r

    m = n + nf
    r0 = residual(np.zeros(m))
    A = np.empty((m, m))
    for j in range(m):
        e = np.zeros(m)
        e[j] = 1.0
        A[:, j] = residual(e) - r0
    x = np.linalg.solve(A, -r0)
    return x[:n]


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("bed", [False, True])
def test_stage_hbar_vs_dense_lu(bc, bed):
    for n in (8, 13, 32):
        U, b = rand_state(n, seed=n + 10 * bc + bed, bed=bed)
        Uo, _ = rand_state(n, seed=100 + n, bed=False)
        lam = 250.0
        p = O.make_params(lam=lam, dx=0.3, bc=bc, has_b=int(bed))
        tau = 0.02
        rc, Un, d = O.stage(p, tau, b, U, Uo, debug=True)
        assert rc == 0
        hb = _uneliminated_hbar(n, p, tau, b, U[0], Uo[0], d)
        assert np.max(np.abs(hb - d["hbar"])) <= 1e-13 * np.max(np.abs(hb))
        assert np.array_equal(Un[0], d["hbar"])


# ---------------------------------------------------------------------------
# Exact relaxation elimination (Sec. 3.1 eq. b1): the oracle's (m, W) must
# satisfy the two implicit equations of the semi-discrete SI system
# (Sec. 4.2 eq. GN_hyp_eq_semi, third and fourth lines, with the bed source).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("bed", [False, True])
def test_relaxation_pair_satisfies_implicit_equations(bed):
    n = 24
    U, b = rand_state(n, seed=3, bed=bed)
    Uo, _ = rand_state(n, seed=4)
    lam, tau, dx = 1e4, 0.01, 0.2
    p = O.make_params(lam=lam, dx=dx, bc=0, has_b=int(bed))
    rc, Un, d = O.stage(p, tau, b, U, Uo, debug=True)
    assert rc == 0
    hb, qn, mn, Wn = Un
    bb = np.zeros(n) if b is None else b
    Db = (np.roll(bb, -1) - np.roll(bb, 1)) / (2 * dx)
    dFm = (d["Fm"][1:] - d["Fm"][:-1]) / dx
    dFW = (d["FW"][1:] - d["FW"][:-1]) / dx
    r_m = mn - (Uo[2] - tau * dFm - tau * 1.5 * U[1] * Db + tau * Wn)
    r_W = Wn - (Uo[3] - tau * dFW - tau * lam * (mn / hb ** 2 - 1.0))
    assert np.max(np.abs(r_m)) < 1e-12 * np.max(np.abs(mn))
    assert np.max(np.abs(r_W)) < 1e-12 * max(1.0, lam * tau)


# ---------------------------------------------------------------------------
# Linearisation coefficients vs the paper's pressure law (Sec. 2.2 eq. hSGN_p)
# along the exact relaxation closure (eq. b1): P0 = P(h_E), beta = dP/dh at
# h_E when eta_E equals the closure's eta; same for p~ and phi (eq. hSGNb_eq).
# ---------------------------------------------------------------------------
def test_coefficients_vs_pressure_law():
    n, g = 6, 9.81
    for lam in (100.0, 1e3, 1e4):
        for hE in (0.3, 1.0, 2.0):
            for eta_ratio in (0.97, 1.0, 1.05):
                tau = 0.01
                mE = eta_ratio * hE * hE
                # uniform periodic state: fluxes cancel; choose W_old so that
                # m-dagger / beta_1 = m_E (closure eta equals eta_E)
                Wold = lam * tau * (mE / hE ** 2 - 1.0)
                U = (np.full(n, hE), np.zeros(n), np.full(n, mE), np.zeros(n))
                Uo = (np.full(n, hE), np.zeros(n), np.full(n, mE), np.full(n, Wold))
                p = O.make_params(lam=lam, dx=0.1, bc=0)
                rc, _, d = O.stage(p, tau, None, U, Uo, debug=True)
                assert rc == 0
                mdag = d["md"][0]

                def mbar(h):
                    return mdag * h * h / (h * h + lam * tau * tau)

                def P(h):
                    mm = mbar(h)
                    return 0.5 * g * h * h + lam / 3.0 * (mm / h) * (1.0 - mm / (h * h))

                def pt(h):
                    return lam / 3.0 * (1.0 - mbar(h) / (h * h))

                eps = 1e-5 * hE
                dP = (P(hE + eps) - P(hE - eps)) / (2 * eps)
                dpt = (pt(hE + eps) - pt(hE - eps)) / (2 * eps)
                assert abs(d["P0"][0] - P(hE)) <= 1e-12 * abs(P(hE))
                assert abs(d["pt0"][0] - pt(hE)) <= 1e-10 * (1 + abs(pt(hE)))
                assert abs(d["beta"][0] - dP) <= 1e-7 * abs(dP)
                assert abs(d["phi"][0] - dpt) <= 1e-7 * (1 + abs(dpt))


# ---------------------------------------------------------------------------
# 0-D relaxation ODE: a uniform periodic state keeps h and q; then
# m_t = W, W_t = lam (1 - m/h^2) (Sec. 2.2 eq. hSGN_eq), solution
# m = h^2 + A cos(w t), w = sqrt(lam)/h.  Second order in dt; L-stable.
# ---------------------------------------------------------------------------
def test_relaxation_ode_second_order_and_damped():
    n, h0, lam, A, T = 4, 1.0, 100.0, 0.01, 1.0
    w = math.sqrt(lam) / h0
    errs = []
    for nsteps in (50, 100, 200, 400):
        p = O.make_params(lam=lam, dx=1.0, bc=0, dt_fixed=T / nsteps)
        U = (np.full(n, h0), np.zeros(n), np.full(n, h0 ** 2 + A), np.zeros(n))
        rc, Un, t = O.run(p, None, U, 0.0, nsteps)
        assert rc == 0
        assert abs(t - T) < 1e-12
        exact = h0 ** 2 + A * math.cos(w * T)
        errs.append(abs(Un[2][0] - exact))
        assert np.max(np.abs(Un[0] - h0)) < 1e-12 and np.max(np.abs(Un[1])) < 1e-12
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(rates) > 1.85, (errs, rates)
    # stiff limit (w dt = 100): the oscillation is damped, not amplified
    p = O.make_params(lam=lam, dx=1.0, bc=0, dt_fixed=10.0)
    U = (np.full(n, h0), np.zeros(n), np.full(n, h0 ** 2 + A), np.zeros(n))
    rc, Un, _ = O.run(p, None, U, 0.0, 3)
    assert rc == 0 and abs(Un[2][0] - h0 ** 2) < 0.05 * A


# ---------------------------------------------------------------------------
# Conservation: periodic mass (divergence form) and flat-bed momentum
# (telescoping face fluxes; the IMEX weights sum to one).
# ---------------------------------------------------------------------------
def test_mass_and_momentum_conservation_periodic():
    wl = WL.solitary(N=800, t_end=0.0, nsteps=100)
    n, prm, b, U = wl.instance(0)
    p = O.make_params(**prm)
    rc, Un, t = O.run(p, b, U, 0.0, 100)
    assert rc == 0
    assert abs(Un[0].sum() - U[0].sum()) <= 1e-13 * U[0].sum()
    assert abs(Un[1].sum() - U[1].sum()) <= 1e-13 * np.abs(U[1]).sum()
    # with a periodic bed mass is still conserved
    x = (np.arange(n) + 0.5) * prm["dx"]
    bed = 0.2 * (1 + np.sin(2 * np.pi * x / (n * prm["dx"])))
    U2 = (U[0] - bed, U[1], (U[0] - bed) ** 2, U[3] * 0)
    p2 = O.make_params(**{**prm, "has_b": 1})
    rc, Un2, _ = O.run(p2, bed, U2, 0.0, 50)
    assert rc == 0
    assert abs(Un2[0].sum() - U2[0].sum()) <= 1e-13 * U2[0].sum()


# ---------------------------------------------------------------------------
# Lake at rest: flat and over the trapezoid bar, lam in {1e2, 1e4}.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lam", [100.0, 1e4])
@pytest.mark.parametrize("bed", [False, True])
def test_lake_at_rest(lam, bed):
    wl = WL.lake_at_rest(N=300, lam=lam, bed=bed)
    n, prm, b, U = wl.instance(0)
    p = O.make_params(**prm)
    rc, Un, t = O.run(p, b, U, 0.0, 100)
    assert rc == 0
    zeta = Un[0] + (b if b is not None else 0.0)
    assert np.max(np.abs(Un[1])) <= 1e-12
    assert np.max(np.abs(zeta - 0.4)) <= 1e-12
    assert np.max(np.abs(Un[2] - Un[0] ** 2)) <= 1e-12
    assert np.max(np.abs(Un[3])) <= 1e-12


# ---------------------------------------------------------------------------
# SGN solitary wave (Sec. 6.3 closed form).
# ---------------------------------------------------------------------------
def test_solitary_wave_config():
    wl = WL.solitary()  # N = 800 on [0, 200], lam = 100, t_end = 10 s
    n, prm, b, U = wl.instance(0)
    p = O.make_params(**prm)
    rc, Un, t = O.run(p, b, U, 0.0, 100000)
    assert rc == 0 and abs(t - 10.0) < 1e-12
    x = (np.arange(n) + 0.5) * prm["dx"]
    he, _, _ = WL.soliton(x, 1.0, 0.2, 100.0, t)
    err = np.abs(Un[0] - he).sum() / np.abs(Un[0]).sum()
    assert err < 6e-4
    crest = x[np.argmax(Un[0])]
    assert abs(crest - (100.0 + WL.soliton_speed(1.0, 0.2) * t)) <= prm["dx"]


@pytest.mark.slow
def test_solitary_error_falls_with_lambda():
    errs = []
    for lam in (10.0, 100.0, 1000.0):
        wl = WL.solitary(N=3200, lam=lam, t_end=3.0)
        n, prm, b, U = wl.instance(0)
        rc, Un, t = O.run(O.make_params(**prm), b, U, 0.0, 100000)
        assert rc == 0
        x = (np.arange(n) + 0.5) * prm["dx"]
        he, _, _ = WL.soliton(x, 1.0, 0.2, 100.0, t)
        errs.append(np.abs(Un[0] - he).sum() / np.abs(Un[0]).sum())
    assert errs[0] / errs[1] > 5 and errs[1] / errs[2] > 5, errs


@pytest.mark.slow
def test_second_order_self_convergence():
    sols = []
    for N in (400, 800, 1600, 3200):
        wl = WL.solitary(N=N, lam=100.0, t_end=3.0)
        n, prm, b, U = wl.instance(0)
        p = O.make_params(**{**prm, "cfl": 0.45})
        rc, Un, t = O.run(p, b, U, 0.0, 100000)
        assert rc == 0
        sols.append(Un[0])
    # restrict fine solutions to the coarsest mesh by cell averaging
    def restrict(a, f):
        return a.reshape(-1, f).mean(1)
    d1 = np.abs(restrict(sols[1], 2) - sols[0]).sum()
    d2 = np.abs(restrict(sols[2], 4) - restrict(sols[1], 2)).sum()
    d3 = np.abs(restrict(sols[3], 8) - restrict(sols[2], 4)).sum()
    r1, r2 = d1 / d2, d2 / d3
    assert r1 > 3.3 and r2 > 3.5, (r1, r2)


# ---------------------------------------------------------------------------
# Linear dispersion of the hSGN system about rest (derived from
# Sec. 2.2 eq. hSGN_eq): w^2 (1 + (lam/3) k^2 / (lam/h0^2 - w^2)) = g h0 k^2.
# A right-going eigenmode is advanced one period; its phase error vanishes
# at second order and converges to this relation (not to SGN or to SW).
# ---------------------------------------------------------------------------
def _omega(k, h0, lam, g=9.81):
    # solve the quadratic in w^2: w^4 - w^2 (lam/h0^2 + lam k^2/3 + g h0 k^2) + g h0 k^2 lam/h0^2 = 0
    B = lam / h0 ** 2 + lam * k * k / 3 + g * h0 * k * k
    Cc = g * h0 * k * k * lam / h0 ** 2
    w2 = 0.5 * (B - math.sqrt(B * B - 4 * Cc))
    return math.sqrt(w2)


def test_linear_dispersion_relation():
    h0, lam, Lw, g = 1.0, 100.0, 10.0, 9.81
    k = 2 * math.pi / Lw
    w = _omega(k, h0, lam)
    w2 = w * w
    assert abs(w2 * (1 + lam / 3 * k * k / (lam / h0 ** 2 - w2)) - g * h0 * k * k) < 1e-12
    eps = 1e-6
    A = (lam / h0) / (lam / h0 ** 2 - w2)
    Tp = 2 * math.pi / w
    phase_err = []
    for N in (32, 64, 128):
        dx = Lw / N
        x = (np.arange(N) + 0.5) * dx
        th = k * x
        hp = eps * np.cos(th)
        mu = A * hp
        U = (h0 + hp, (w / k) * hp, h0 ** 2 + h0 * hp + mu, w * A * eps * np.sin(th))
        nsteps = 4 * N
        p = O.make_params(lam=lam, dx=dx, bc=0, dt_fixed=Tp / nsteps)
        rc, Un, t = O.run(p, None, U, 0.0, nsteps)
        assert rc == 0
        d = Un[0] - h0
        c_ = (d * np.cos(th)).sum()
        s_ = (d * np.sin(th)).sum()
        phase_err.append(math.atan2(s_, c_))  # zero for an exact period
    r1 = abs(phase_err[0] / phase_err[1])
    r2 = abs(phase_err[1] / phase_err[2])
    assert r1 > 3.5 and r2 > 3.5, phase_err
    # the Richardson-extrapolated phase error must be far below the phase gap
    # between the hSGN relation and the SGN relation it tends to
    wsgn = math.sqrt(g * h0 * k * k / (1 + k * k * h0 * h0 / 3))
    gap = abs(w - wsgn) / w * 2 * math.pi
    ext = (4 * phase_err[2] - phase_err[1]) / 3
    assert abs(ext) < 0.01 * gap, (ext, gap)


# ---------------------------------------------------------------------------
# Complex-step build of the oracle (reference for the adjoint): it returns
# the double build's loss in its real part and, for a perturbation i*eps*v,
# the directional derivative in its imaginary part; checked against central
# differences of the double build with Richardson extrapolation.
# ---------------------------------------------------------------------------
def test_complex_step_build_differentiates_the_oracle():
    wl = WL.batched_bar(n_inst=1, seed=5, n_lo=300, n_hi=300)
    n, prm, b, U0 = wl.instance(0)
    prm = dict(prm, dt_fixed=0.004, lam=1000.0)
    p = O.make_params(**prm)
    g = np.array([n // 4, n // 2, 3 * n // 4])
    tgt = np.full((15, 3), 0.41)
    zeta = U0[0] + b
    rng = np.random.default_rng(1)

    def state(z, bb):
        h = z - bb
        return (h, np.zeros(n), h * h, np.zeros(n))

    _, J0, _ = O.run_loss(p, b, state(zeta, b), 15, g, tgt)
    for kind in ("zeta", "b"):
        v = rng.standard_normal(n) * 1e-3
        eps = 1e-30
        if kind == "zeta":
            rc, Jc = O.run_loss_cs(p, b.astype(complex), state(zeta + 1j * eps * v, b.astype(complex)), 15, g, tgt)
            f = lambda e: O.run_loss(p, b, state(zeta + e * v, b), 15, g, tgt)[1]
        else:
            bc = b + 1j * eps * v
            rc, Jc = O.run_loss_cs(p, bc, state(zeta.astype(complex), bc), 15, g, tgt)
            f = lambda e: O.run_loss(p, b + e * v, state(zeta, b + e * v), 15, g, tgt)[1]
        assert rc == 0
        assert abs(Jc.real - J0) <= 1e-14 * abs(J0)
        d_cs = Jc.imag / eps
        fd = lambda e: (f(e) - f(-e)) / (2 * e)
        d_rich = (4 * fd(1e-4) - fd(2e-4)) / 3
        assert abs(d_cs - d_rich) <= 1e-7 * abs(d_cs), (kind, d_cs, d_rich)


def test_gauge_series_consistent_with_run_and_loss():
    """The recorded gauge series is the state the plain run reaches, and its
    misfit against any targets is the loss the loss routine accumulates."""
    wl = WL.batched_bar(n_inst=1, seed=6, n_lo=200, n_hi=200)
    n, prm, b, U0 = wl.instance(0)
    prm = dict(prm, dt_fixed=0.005)
    p = O.make_params(**prm)
    g = np.array([3, n // 2, n - 1])
    rc, ser = O.run_gauges(p, b, U0, 9, g)
    assert rc == 0 and ser.shape == (9, 3)
    for k in (1, 4, 9):
        _, Uk, _ = O.run(p, b, U0, 0.0, k)
        assert np.array_equal(ser[k - 1], Uk[0][g])
    tgt = np.random.default_rng(2).uniform(0.3, 0.5, size=(9, 3))
    _, J, _ = O.run_loss(p, b, U0, 9, g, tgt)
    assert J == pytest.approx(0.5 * np.sum((ser - tgt) ** 2), rel=1e-14)


# ---------------------------------------------------------------------------
# First-order scheme (Sec. 4.2 as printed: one stage with tau = dt, cell
# values at the faces): first-order self-convergence, conservation, lake
# at rest, and the two-stage step's results untouched by the order switch.
# ---------------------------------------------------------------------------
def test_first_order_self_convergence():
    sols = []
    for N in (400, 800, 1600, 3200):
        wl = WL.solitary(N=N, lam=100.0, t_end=3.0)
        n, prm, b, U = wl.instance(0)
        p = O.make_params(**{**prm, "cfl": 0.45, "order": 1})
        rc, Un, t = O.run(p, b, U, 0.0, 100000)
        assert rc == 0 and abs(t - 3.0) < 1e-12
        sols.append(Un[0])

    def restrict(a, f):
        return a.reshape(-1, f).mean(1)
    d1 = np.abs(restrict(sols[1], 2) - sols[0]).sum()
    d2 = np.abs(restrict(sols[2], 4) - restrict(sols[1], 2)).sum()
    d3 = np.abs(restrict(sols[3], 8) - restrict(sols[2], 4)).sum()
    r1, r2 = d1 / d2, d2 / d3
    # ratios approach 2 from below (1.56, 1.69, then 1.81 at 6400 cells):
    # first order, pre-asymptotic; a second-order scheme gives ~4 here
    assert 1.4 < r1 < r2 < 2.2, (r1, r2)


def test_first_order_conserves_and_keeps_rest():
    wl = WL.solitary(N=600, t_end=0.0, nsteps=50)
    n, prm, b, U = wl.instance(0)
    p = O.make_params(**{**prm, "order": 1})
    rc, Un, t = O.run(p, b, U, 0.0, 50)
    assert rc == 0
    assert abs(Un[0].sum() - U[0].sum()) <= 1e-13 * U[0].sum()
    assert abs(Un[1].sum() - U[1].sum()) <= 1e-13 * np.abs(U[1]).sum()
    for lam in (100.0, 1e4):
        wl = WL.lake_at_rest(N=300, lam=lam, bed=True)
        n, prm, b, U = wl.instance(0)
        rc, Un, t = O.run(O.make_params(**{**prm, "order": 1}), b, U, 0.0, 100)
        assert rc == 0
        assert np.max(np.abs(Un[1])) <= 1e-12
        assert np.max(np.abs(Un[0] + b - 0.4)) <= 1e-12


def test_first_order_step_is_one_full_stage():
    """order 1 = or_stage with tau = dt and U_E = U_old = U^n; the
    reconstruction switch reaches the fluxes (the two orders differ)."""
    wl = WL.batched_bar(n_inst=1, seed=8, n_lo=300, n_hi=300)
    n, prm, b, U = wl.instance(0)
    p1 = O.make_params(**{**prm, "order": 1})
    rc, U1, t1, dt = O.step(p1, b, U, 0.0)
    assert rc == 0 and dt > 0
    rc, Us = O.stage(p1, dt, b, U, U)
    assert rc == 0
    for a, c in zip(U1, Us):
        assert np.array_equal(a, c)
    p2 = O.make_params(**prm)
    rc, Uf = O.stage(p2, dt, b, U, U)
    assert max(np.max(np.abs(a - c)) for a, c in zip(Uf, Us)) > 1e-6


# ---------------------------------------------------------------------------
# Fully explicit hSGN scheme with Heun's method (Sec. 4.1, scheme 1, flat
# bottom; Rusanov fluxes with speed |u| + c on all four fields).
# ---------------------------------------------------------------------------
EX = O.SCHEME_EXPLICIT


@pytest.mark.parametrize("bc", [0, 1])
def test_explicit_lake_at_rest(bc):
    n = 64
    h = np.full(n, 0.7)
    U = (h, np.zeros(n), h * h, np.zeros(n))
    for lam in (100.0, 1e4):
        p = O.make_params(lam=lam, dx=0.05, cfl=0.4, bc=bc, scheme=EX)
        rc, Un, t = O.run(p, None, U, 0.0, 200)
        assert rc == 0 and t > 0
        for a, b in zip(U, Un):
            assert np.array_equal(a, b)


def test_explicit_heun_on_uniform_state():
    """A uniform state has no spatial terms: h' = 0, q' = 0, m' = W,
    W' = -lambda (m / h^2 - 1).  One Heun step of this affine system is its
    second-order Taylor polynomial y + dt f + dt^2/2 A f (A = df/dy)."""
    n, h0, q0, m0, W0, lam, dt = 16, 0.8, 0.3, 0.7, 0.2, 500.0, 1e-3
    U = tuple(np.full(n, v) for v in (h0, q0, m0, W0))
    p = O.make_params(lam=lam, dx=0.1, bc=0, dt_fixed=dt, scheme=EX)
    rc, Un, t, dt_used = O.step(p, None, U)
    assert rc == 0 and dt_used == dt
    fm, fW = W0, -lam * (m0 / h0 ** 2 - 1.0)
    Afm, AfW = fW, -lam / h0 ** 2 * fm
    m2 = m0 + dt * fm + 0.5 * dt * dt * Afm
    W2 = W0 + dt * fW + 0.5 * dt * dt * AfW
    assert np.all(Un[0] == h0) and np.all(Un[1] == q0)
    assert np.max(np.abs(Un[2] - m2)) < 1e-15 and np.max(np.abs(Un[3] - W2)) < 1e-13


def test_semi_implicit_dt_rule():
    """dt = CFL dx / max(|u| + sqrt(g h)), capped so that max|u| dt / dx <=
    MCFL (Sec. 5), replaced by a fixed step when one is given, and clamped
    to t_end (0 once t_end is reached): each branch made to bind."""
    g, dx, cfl, mcfl = 9.81, 0.1, 0.9, 0.5
    # subcritical: the CFL rule binds
    h = np.array([1.0, 0.5, 2.0])
    q = np.array([0.2, -0.4, 0.1])
    p = O.make_params(dx=dx, cfl=cfl, mcfl=mcfl)
    s = max(abs(q[i] / h[i]) + math.sqrt(g * h[i]) for i in range(3))
    assert abs(O.dt(p, h, q) - cfl * dx / s) < 1e-17
    # supercritical: the material cap binds (max|u| = 6, c ~ 1)
    h = np.array([0.1, 0.1, 0.1])
    q = np.array([0.5, -0.6, 0.1])
    s = max(abs(q[i] / h[i]) + math.sqrt(g * h[i]) for i in range(3))
    assert 6.0 * (cfl * dx / s) / dx > mcfl
    assert abs(O.dt(p, h, q) - mcfl * dx / 6.0) < 1e-17
    # no cap when mcfl <= 0
    p0 = O.make_params(dx=dx, cfl=cfl, mcfl=0.0)
    assert abs(O.dt(p0, h, q) - cfl * dx / s) < 1e-17
    # a fixed step is taken as given
    pf = O.make_params(dx=dx, cfl=cfl, mcfl=mcfl, dt_fixed=0.0123)
    assert O.dt(pf, h, q) == 0.0123
    # t_end: the last step is shortened, then the state is frozen
    pt = O.make_params(dx=dx, cfl=cfl, mcfl=mcfl, dt_fixed=0.0123, t_end=0.05)
    assert O.dt(pt, h, q, t=0.045) == pytest.approx(0.005, abs=1e-16)
    assert O.dt(pt, h, q, t=0.05) == 0.0


def test_explicit_dt_rule():
    """dt = CFL dx / max(|u| + c), c^2 = g h + (lambda/3)(eta/h)^2 (Sec. 5,
    eq. CFL_ex), clamped to t_end."""
    h = np.array([1.0, 0.5, 2.0])
    q = np.array([0.2, -0.4, 0.1])
    m = np.array([1.1, 0.2, 4.4])
    lam, g, dx, cfl = 300.0, 9.81, 0.1, 0.4
    p = O.make_params(lam=lam, dx=dx, cfl=cfl, scheme=EX)
    mu = max(abs(q[i] / h[i]) + math.sqrt(g * h[i] + lam / 3 * (m[i] / h[i] ** 2) ** 2) for i in range(3))
    assert abs(O.dt_ex(p, h, q, m) - cfl * dx / mu) < 1e-17
    p2 = O.make_params(lam=lam, dx=dx, cfl=cfl, t_end=0.01, scheme=EX)
    assert O.dt_ex(p2, h, q, m, t=0.0095) == pytest.approx(0.0005, abs=1e-15)


def test_explicit_conserves_mass_and_is_mirror_symmetric():
    (h, q, m, W), _ = rand_state(128, 21, amp=0.1)
    p = O.make_params(lam=300.0, dx=0.05, cfl=0.4, bc=0, scheme=EX)
    rc, Un, t = O.run(p, None, (h, q, m, W), 0.0, 50)
    assert rc == 0
    assert abs(Un[0].sum() - h.sum()) / h.sum() < 1e-14
    # x -> -x: h, m, W even, q odd; cell i <-> cell n - 1 - i
    rcm, Um, tm = O.run(p, None, (h[::-1].copy(), -q[::-1].copy(), m[::-1].copy(), W[::-1].copy()),
                        0.0, 50)
    assert rcm == 0 and tm == t
    for a, b, s in zip(Un, Um, (1, -1, 1, 1)):
        assert np.max(np.abs(a - s * b[::-1])) < 1e-12 * max(1.0, np.max(np.abs(a)))


def test_explicit_rest_state_is_linearly_stable():
    """Spectral radius of one step's Jacobian at rest (central differences of
    the oracle): at most 1 to the accuracy of the differences, for CFL 0.4."""
    N = 32
    h = np.ones(N)
    z = np.zeros(N)
    for lam in (100.0, 1000.0):
        p = O.make_params(lam=lam, dx=0.04, cfl=0.4, bc=0, scheme=EX)
        eps = 1e-6
        J = np.zeros((4 * N, 4 * N))
        for k in range(4 * N):
            Up = [h.copy(), z.copy(), h * h, z.copy()]
            Um = [h.copy(), z.copy(), h * h, z.copy()]
            Up[k // N][k % N] += eps
            Um[k // N][k % N] -= eps
            J[:, k] = (np.concatenate(O.step(p, None, Up)[1]) - np.concatenate(O.step(p, None, Um)[1])) / (2 * eps)
        rho = np.max(np.abs(np.linalg.eigvals(J)))
        assert rho < 1 + 1e-7, (lam, rho)


def test_explicit_converges_to_the_semi_implicit_solution():
    """Both schemes discretise the same hSGN system to second order, so their
    difference at a fixed time falls like dx^2 (solitary wave, lambda = 100)."""
    diffs = []
    for N in (200, 400, 800):
        wl = WL.solitary(N=N, L=100.0, h0=1.0, a=0.2, lam=100.0, t_end=1.0)
        n, prm, b, U = wl.instance(0)
        rce, Ue, te = O.run(O.make_params(**{**prm, "cfl": 0.4}, scheme=EX), None, U, 0.0, 100000)
        rcs, Us, ts = O.run(O.make_params(**prm), None, U, 0.0, 100000)
        assert rce == 0 and rcs == 0 and te == 1.0 and ts == 1.0
        diffs.append(np.sum(np.abs(Ue[0] - Us[0])) * prm["dx"])
    r1, r2 = math.log2(diffs[0] / diffs[1]), math.log2(diffs[1] / diffs[2])
    assert 1.8 < r1 < 2.4 and 1.8 < r2 < 2.4, diffs


def test_explicit_linear_dispersion_relation():
    """A small sinusoid propagates with the hSGN linear phase speed; the phase
    error after one period falls at second order and its extrapolation is far
    below the gap to the SGN relation (as for the semi-implicit scheme)."""
    h0, lam, Lw, g = 1.0, 100.0, 10.0, 9.81
    k = 2 * math.pi / Lw
    w = _omega(k, h0, lam)
    eps = 1e-6
    A = (lam / h0) / (lam / h0 ** 2 - w * w)
    Tp = 2 * math.pi / w
    phase_err = []
    for N in (32, 64, 128):
        dx = Lw / N
        x = (np.arange(N) + 0.5) * dx
        th = k * x
        hp = eps * np.cos(th)
        U = (h0 + hp, (w / k) * hp, h0 ** 2 + h0 * hp + A * hp, w * A * eps * np.sin(th))
        nsteps = 8 * N
        p = O.make_params(lam=lam, dx=dx, bc=0, dt_fixed=Tp / nsteps, scheme=EX)
        rc, Un, t = O.run(p, None, U, 0.0, nsteps)
        assert rc == 0
        d = Un[0] - h0
        phase_err.append(math.atan2((d * np.sin(th)).sum(), (d * np.cos(th)).sum()))
    r1 = abs(phase_err[0] / phase_err[1])
    r2 = abs(phase_err[1] / phase_err[2])
    assert r1 > 3.5 and r2 > 3.5, phase_err
    wsgn = math.sqrt(g * h0 * k * k / (1 + k * k * h0 * h0 / 3))
    gap = abs(w - wsgn) / w * 2 * math.pi
    ext = (4 * phase_err[2] - phase_err[1]) / 3
    assert abs(ext) < 0.01 * gap, (ext, gap)


def test_explicit_rejects_a_bed():
    n = 16
    h = np.full(n, 0.5)
    p = O.make_params(lam=100.0, dx=0.1, has_b=1, scheme=EX)
    rc, _, _, _ = O.step(p, np.zeros(n), (h, np.zeros(n), h * h, np.zeros(n)))
    assert rc == O.EINVAL


# ---------------------------------------------------------------------------
# Standard SGN equations, elliptic-hyperbolic form (Sec. 4.3-4.4, scheme 2,
# flat bottom, Heun's method).
# ---------------------------------------------------------------------------
SGN = O.SCHEME_SGN


@pytest.mark.parametrize("bc", [0, 1])
def test_sgn_rest_and_uniform_flow_are_steady(bc):
    n = 48
    for u0 in (0.0, 0.3):
        h = np.full(n, 0.6)
        U = (h, u0 * h, h * h, np.zeros(n))
        p = O.make_params(dx=0.05, bc=bc, scheme=SGN)
        rc, Un, t = O.run(p, None, U, 0.0, 100)
        assert rc == 0 and t > 0
        for a, b in zip(U, Un):
            assert np.array_equal(a, b)


def test_sgn_conserves_mass_and_momentum_periodic():
    """Periodic: the Rusanov fluxes telescope, and sum_i h_i phi_i equals the
    sum of the right-hand side h*, itself a telescoping difference."""
    (h, q, m, W), _ = rand_state(200, 31, amp=0.1)
    p = O.make_params(dx=0.05, bc=0, scheme=SGN)
    rc, Un, t = O.run(p, None, (h, q, m, W), 0.0, 100)
    assert rc == 0
    assert abs(Un[0].sum() - h.sum()) / h.sum() < 1e-14
    assert abs(Un[1].sum() - q.sum()) / np.abs(q).sum() < 1e-13
    assert np.array_equal(Un[2], m) and np.array_equal(Un[3], W)


def _sgn_phi_spectral(h, u, L, g=9.81):
    """The continuous elliptic problem of eq. SGN_standard,
    h phi - (h^3/3 phi_x)_x = -(h^3/3 g h_xx + 2 h^3/3 u_x^2)_x, periodic,
    by Fourier collocation (a dense solve): spectrally accurate."""
    N = len(h)
    k = 2 * np.pi * np.fft.fftfreq(N, d=L / N)
    I = np.eye(N)
    D = np.real(np.fft.ifft(1j * k[:, None] * np.fft.fft(I, axis=0), axis=0))
    hx, hxx, ux = D @ h, D @ (D @ h), D @ u
    rhs = -D @ (h ** 3 / 3 * g * hxx + 2 * h ** 3 / 3 * ux ** 2)
    A = np.diag(h) - D @ np.diag(h ** 3 / 3) @ D
    return np.linalg.solve(A, rhs)


def test_sgn_phi_converges_to_the_continuous_elliptic_problem():
    L = 10.0
    errs = []
    for N in (64, 128, 256):
        x = (np.arange(N) + 0.5) * (L / N)
        h = 1.0 + 0.2 * np.sin(2 * np.pi * x / L) + 0.05 * np.cos(4 * np.pi * x / L)
        u = 0.3 * np.cos(2 * np.pi * x / L)
        rc, phi = O.sgn_phi(O.make_params(dx=L / N, bc=0, scheme=SGN), h, h * u)
        assert rc == 0
        ref = _sgn_phi_spectral(h, u, L)
        errs.append(np.max(np.abs(phi - ref)) / np.max(np.abs(ref)))
    assert errs[0] / errs[1] > 3.6 and errs[1] / errs[2] > 3.6, errs
    assert errs[2] < 2e-3


def test_sgn_solitary_wave_second_order():
    """The SGN solitary wave is an exact travelling solution (Sec. 6.3):
    the error at t = 2 s falls like dx^2."""
    L, errs = 100.0, []
    for N in (200, 400, 800):
        wl = WL.solitary(N=N, L=L, h0=1.0, a=0.2, lam=100.0, t_end=2.0)
        n, prm, b, U = wl.instance(0)
        rc, Un, t = O.run(O.make_params(**prm, scheme=SGN), None, U, 0.0, 100000)
        assert rc == 0 and t == 2.0
        x = (np.arange(N) + 0.5) * (L / N)
        he, _, _ = WL.soliton(x, 1.0, 0.2, 0.5 * L, t=t)
        errs.append(np.sum(np.abs(Un[0] - he)) * L / N)
    r1, r2 = math.log2(errs[0] / errs[1]), math.log2(errs[1] / errs[2])
    assert 1.8 < r1 < 2.3 and 1.8 < r2 < 2.3, errs


def test_sgn_linear_dispersion_relation():
    """A small sinusoid moves with the SGN phase speed,
    w^2 = g h k^2 / (1 + k^2 h^2 / 3); the phase error after one period falls
    at second order and extrapolates far below the gap to shallow water."""
    h0, Lw, g = 1.0, 10.0, 9.81
    k = 2 * math.pi / Lw
    w = math.sqrt(g * h0 * k * k / (1 + k * k * h0 * h0 / 3))
    eps = 1e-6
    Tp = 2 * math.pi / w
    phase_err = []
    for N in (32, 64, 128):
        dx = Lw / N
        x = (np.arange(N) + 0.5) * dx
        th = k * x
        hp = eps * np.cos(th)
        U = (h0 + hp, (w / k) * hp, np.ones(N), np.zeros(N))
        nsteps = 4 * N
        p = O.make_params(dx=dx, bc=0, dt_fixed=Tp / nsteps, scheme=SGN)
        rc, Un, t = O.run(p, None, U, 0.0, nsteps)
        assert rc == 0
        d = Un[0] - h0
        phase_err.append(math.atan2((d * np.sin(th)).sum(), (d * np.cos(th)).sum()))
    assert abs(phase_err[0] / phase_err[1]) > 3.5 and abs(phase_err[1] / phase_err[2]) > 3.5, phase_err
    gap = abs(math.sqrt(g * h0) * k - w) / w * 2 * math.pi
    ext = (4 * phase_err[2] - phase_err[1]) / 3
    assert abs(ext) < 0.01 * gap, (ext, gap)
