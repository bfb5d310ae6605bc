"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bar, per instance, after the given number of steps:
 (1) state: max over fields and cells of |gpu - oracle| divided by max over
     fields and cells of |oracle| <= 1e-11 (relative error of the state);
 (2) every field f: max |gpu_f - oracle_f| <= max(1e-11 max |oracle_f|,
     8 d_f), where d_f is how far the oracle's own f moves when its initial
     state is perturbed by 2^-53 relative (its rounding sensitivity).  On the
     stiff instances (lambda >= 1e3 over the bar) W = h w is the difference
     of two O(lambda tau) terms, and a half-ulp input perturbation already
     moves it by 2e-11 relative to max |W| after 100 steps.
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_2510_07539_amd import workloads as WL  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-11


def _solver():
    from paper_2510_07539_amd.hsgn import Solver
    return Solver


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def field_err(a, ref):
    scale = np.max(np.abs(ref))
    d = np.max(np.abs(a - ref)) if len(ref) else 0.0
    return d / scale if scale > 0 else d


def check_instance(j, U, wl, nsteps, tol=TOL, seed=0, state_sens=False, order=2, scheme=0,
                   cfl=None):
    """Bars (1) and (2) for instance j; returns (state error, worst field ratio).
    state_sens: bar (1) becomes max(tol, 8 s) with s the oracle's own relative
    state sensitivity to a half-ulp perturbation (for runs that approach a
    loss of coercivity, where that sensitivity itself exceeds tol)."""
    n, prm, b, U0 = wl.instance(j)
    if cfl is not None:
        prm = dict(prm, cfl=cfl)
    p = O.make_params(**prm, order=order, scheme=scheme)
    orc, Uo, to = O.run(p, b, U0, 0.0, nsteps)
    assert orc == 0, ("oracle", j, orc)
    rng = np.random.default_rng(seed + j)
    Up0 = tuple(u * (1.0 + 2.0 ** -53 * rng.choice([-1.0, 1.0], size=n)) for u in U0)
    _, Up, _ = O.run(p, b, Up0, 0.0, nsteps)
    o0, o1 = int(wl.offsets[j]), int(wl.offsets[j + 1])
    scale = max(np.max(np.abs(x)) for x in Uo)
    dev = [np.max(np.abs(U[f][o0:o1] - Uo[f])) for f in range(4)]
    state_err = max(dev) / scale
    state_tol = tol
    if state_sens:
        s_own = max(np.max(np.abs(Up[f] - Uo[f])) for f in range(4)) / scale
        state_tol = max(tol, 8.0 * s_own)
    assert state_err <= state_tol, ("instance", j, "state", state_err, state_tol)
    worst = 0.0
    for f in range(4):
        sens = np.max(np.abs(Up[f] - Uo[f]))
        bound = max(tol * np.max(np.abs(Uo[f])), 8.0 * sens, 1e-300)
        assert dev[f] <= bound, ("instance", j, "field", "hqmW"[f], dev[f], bound, sens)
        worst = max(worst, dev[f] / bound)
    return state_err, worst, to


def compare(wl, nsteps, use_run=False, block=50, insts=None, tol=TOL, label="", solver="auto",
            order=2, scheme=0, cfl=None, state_sens=False, margin=None, retry=False):
    note("parity %s [%s, order %d, scheme %d]: %s, %d instances, %d cells, %d steps" % (
        label, solver, order, scheme, wl.name, wl.n_inst, wl.n_cells, nsteps))
    Solver = _solver()
    s = Solver.from_workload(wl, solver=solver, order=order, scheme=scheme, cfl=cfl)
    if margin is not None:
        s.set_halo_margin(margin)
    if retry:
        s.set_halo_retry(True)
    info = s.plan_info()
    note("  plan: %d windows, %d two-pass tiles, halo max %d" % (
        info["windows"], info["exact_tiles"], int(info["halo"].max())))
    if use_run:
        s.run(nsteps, block=block)
    else:
        s.step(nsteps)
    (h, q, m, W), t = s.get_state()
    rc, flags = s.status()
    assert rc == 0, ("status", rc, np.nonzero(flags))
    if margin is not None or retry:
        mg, nr = s.halo_state()
        note("  halo margins %.3g .. %.3g, blocks run again %d" % (mg.min(), mg.max(), nr))
    U = [x.cpu().numpy() for x in (h, q, m, W)]
    tg = t.cpu().numpy()
    s.close()
    insts = range(wl.n_inst) if insts is None else insts
    worst = 0.0
    worst_ratio = 0.0
    for j in insts:
        e, r, to = check_instance(j, U, wl, nsteps, tol, order=order, scheme=scheme, cfl=cfl,
                                  state_sens=state_sens)
        assert abs(tg[j] - to) <= 1e-12 * max(1.0, abs(to)), (j, tg[j], to)
        worst = max(worst, e)
        worst_ratio = max(worst_ratio, r)
    note("  worst state deviation %.3e, worst field deviation / bound %.3f" % (worst, worst_ratio))
    return worst


SOLVERS = ["auto", "exact", "auto_small"]


@pytest.mark.parametrize("solver", SOLVERS)
def test_solitary_single_tile_100_steps(solver):
    compare(WL.solitary(N=800, t_end=0.0), 100, label="C1 geometry", solver=solver)


def test_solitary_to_t_end():
    # the full solitary-wave configuration: t_end = 10 s (about 178 steps)
    wl = WL.solitary()
    compare(wl, 200, label="C1 to t_end")


def test_supercritical_flow_material_cfl_cap():
    """Froude-6 flow over h = 0.1 m (|u| = 6 m/s): the material CFL cap
    max|u| dt / dx <= 0.5 binds instead of the CFL rule on |u| + sqrt(g h)
    (checked on the oracle first); periodic and transmissive, 2 tiles."""
    parts = []
    for bc in (0, 1):
        n, dx = 3000, 0.04
        x = (np.arange(n) + 0.5) * dx
        h = 0.1 * (1.0 + 0.05 * np.sin(2 * np.pi * x / (n * dx)))
        u = np.full(n, 6.0)
        parts.append(WL._part(n, dx, 100.0, bc, h, u, np.zeros(n)))
    wl = WL._pack("supercritical", parts, 30)
    for j in range(wl.n_inst):
        n, prm, b, U0 = wl.instance(j)
        p = O.make_params(**prm)
        umax = float(np.max(np.abs(U0[1] / U0[0])))
        assert O.dt(p, U0[0], U0[1]) == pytest.approx(prm["mcfl"] * prm["dx"] / umax, rel=1e-15)
    compare(wl, 30, label="supercritical (material CFL cap)")


@pytest.mark.parametrize("solver", SOLVERS)
def test_multi_tile_periodic(solver):
    compare(WL.solitary(N=5000, L=1250.0, lam=1000.0, t_end=0.0), 100, label="periodic 3 tiles",
            solver=solver)


@pytest.mark.parametrize("solver", SOLVERS)
def test_dam_break_transmissive_multi_tile(solver):
    compare(WL.dam_break(), 100, label="C2 100 steps", solver=solver)


@pytest.mark.parametrize("solver", SOLVERS)
def test_batched_bar_small_batch(solver):
    wl = WL.batched_bar(n_inst=16, seed=5, n_lo=512, n_hi=9000)
    compare(wl, 100, label="bar batch", solver=solver)


def test_graph_run_matches_step_bitwise():
    Solver = _solver()
    wl = WL.concat("mix", [WL.solitary(N=3000, L=750.0, t_end=0.0),
                           WL.batched_bar(n_inst=3, seed=2, n_lo=700, n_hi=5000)])
    s1 = Solver.from_workload(wl)
    s1.step(60)
    s2 = Solver.from_workload(wl)
    s2.run(60, block=20)
    (a, ta), (b, tb) = s1.get_state(), s2.get_state()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    assert torch.equal(ta, tb)
    # several replays of the cached graph, with eager work in between
    s2.step(3)
    s2.run(40, block=20)
    s1.step(43)
    (a, _), (b, _) = s1.get_state(), s2.get_state()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


@pytest.mark.parametrize("scheme", [0, 1])
def test_graph_cached_across_set_state(scheme):
    """Loading a state whose plan has the same launch configuration keeps the
    captured graph; its replays match a fresh context's eager steps."""
    Solver = _solver()
    wl = WL.concat("mix", [WL.solitary(N=3000, L=750.0, t_end=0.0),
                           WL.solitary(N=700, L=175.0, lam=1000.0, t_end=0.0)])
    kw = dict(scheme=scheme, cfl=0.4 if scheme else None)
    s1 = Solver.from_workload(wl, **kw)
    s1.run(20, block=10)
    s1.set_state(*[torch.from_numpy(a).cuda() for a in wl.state()])
    s1.run(30, block=10)
    s2 = Solver.from_workload(wl, **kw)
    s2.step(30)
    (a, ta), (b, tb) = s1.get_state(), s2.get_state()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    assert torch.equal(ta, tb)
    s1.close()
    s2.close()


@pytest.mark.parametrize("solver", SOLVERS)
def test_edge_sizes_and_frozen_instances(solver):
    parts = []
    for n in (4, 5, 7, 9, 31, 513, 2047, 2048, 2049, 4097):
        for bc in (0, 1):
            parts.append(WL.solitary(N=n, L=0.25 * n, lam=300.0, t_end=0.0, bc=bc,
                                     x0=0.125 * n))
    # an instance that reaches t_end after a few steps, then stays frozen
    parts.append(WL.solitary(N=600, L=150.0, lam=100.0, t_end=0.2))
    # fixed time step
    fixed = WL.solitary(N=1000, L=250.0, lam=100.0, t_end=0.0)
    fixed.dt_fixed[:] = 0.01
    parts.append(fixed)
    parts.append(WL.lake_at_rest(N=700, lam=1e4, bed=True))
    for n in (4095, 4096, 4097, 8300):
        parts.append(WL.solitary(N=n, L=0.25 * n, lam=1e4, t_end=0.0, bc=1, x0=0.125 * n))
        parts.append(WL.solitary(N=n, L=0.25 * n, lam=1e4, t_end=0.0, bc=0, x0=0.125 * n))
    wl = WL.concat("edges", parts)
    compare(wl, 30, label="edge sizes", solver=solver)


def test_lake_at_rest_gpu():
    Solver = _solver()
    for lam in (100.0, 1e4):
        wl = WL.lake_at_rest(N=3000, lam=lam, bed=True)
        s = Solver.from_workload(wl)
        s.step(100)
        (h, q, m, W), _ = s.get_state()
        b = torch.from_numpy(wl.b).to(h.device)
        assert float((h + b - 0.4).abs().max()) <= 1e-12
        assert float(q.abs().max()) <= 1e-12
        assert float(W.abs().max()) <= 1e-12


def test_nonphysical_state_is_flagged_and_frozen():
    from paper_2510_07539_amd.hsgn import HSGN_ENONPHYS, lib
    Solver = _solver()
    wl = WL.concat("bad", [WL.solitary(N=400, L=100.0, t_end=0.0),
                           WL.solitary(N=400, L=100.0, t_end=0.0)])
    wl.h[wl.offsets[1] + 10] = -0.5  # negative depth in the second instance
    s = Solver.from_workload(wl)
    s.step(3)
    rc, flags = s.status()
    assert rc == HSGN_ENONPHYS and flags[1] != 0 and flags[0] == 0
    # the message names the instance, the step in which it was flagged and
    # how many instances carry the flag
    msg = lib().hsgn_last_error(s._h).decode()
    note("  " + msg)
    assert "instance 1:" in msg and "in step 1 " in msg and "1 instance(s)" in msg, msg
    (h, q, m, W), t = s.get_state()
    # the healthy instance still matches the oracle
    U = [x.cpu().numpy() for x in (h, q, m, W)]
    check_instance(0, U, wl, 3)


@pytest.mark.parametrize("solver", SOLVERS)
def test_long_periodic_scaled(solver):
    wl = WL.long_periodic(N=1 << 16)
    compare(wl, 20, label="long periodic scaled", solver=solver)


@pytest.mark.parametrize("solver,margin", [(m, None) for m in SOLVERS] + [("auto_small", 1.0)])
def test_batched_full_size_sampled(solver, margin):
    """The full batched workload (4096 instances) in the launch configuration
    the benchmark times (graph-captured blocks; the autotuner keeps
    auto_small there, at halo margin 1 with the halo retry), and in the
    three solver modes at the default margin; instances sampled for the
    oracle: the smallest and largest, both ends of the batch, the first of
    each lambda, and the longest instance of each lambda (the most
    windows)."""
    wl = WL.batched_bar()
    sizes = wl.sizes()
    pick = [int(np.argmin(sizes)), int(np.argmax(sizes)), 0, 1, 2047, 4095]
    lam = wl.lam
    for v in (100.0, 1000.0, 10000.0):
        sel = np.nonzero(lam == v)[0]
        pick.append(int(sel[0]))
        pick.append(int(sel[np.argmax(sizes[sel])]))
    compare(wl, 100, use_run=True, block=100, insts=sorted(set(pick)),
            label="C3 full, sampled", solver=solver, margin=margin, retry=margin is not None)


def test_default_auxiliary_variables():
    """hsgn_set_state without m and W: m = h^2 and W = -h^2 u_x with the
    central difference of u = q/h (periodic wrap; transmissive ends take the
    boundary cell's own u), on one periodic and one transmissive instance."""
    Solver = _solver()
    wl = WL.concat("defaults", [WL.solitary(N=700, L=175.0, t_end=0.0),
                                WL.dam_break(N=900, xa=-30.0, xb=30.0)])
    wl.q[:] = 0.05 * np.sin(np.arange(wl.n_cells) * 0.37) * wl.h
    s = Solver.from_workload(wl)
    h, q = torch.from_numpy(wl.h).cuda(), torch.from_numpy(wl.q).cuda()
    s.set_state(h, q)
    (h2, q2, m2, W2), _ = s.get_state()
    s.close()
    m2, W2 = m2.cpu().numpy(), W2.cpu().numpy()
    for j in range(wl.n_inst):
        o0, o1 = int(wl.offsets[j]), int(wl.offsets[j + 1])
        hh, uu = wl.h[o0:o1], wl.q[o0:o1] / wl.h[o0:o1]
        if wl.bc[j] == WL.BC_PERIODIC:
            up, um = np.roll(uu, -1), np.roll(uu, 1)
        else:
            up = np.concatenate([uu[1:], uu[-1:]])
            um = np.concatenate([uu[:1], uu[:-1]])
        W = -hh * hh * (up - um) / (2.0 * wl.dx[j])
        assert np.max(np.abs(m2[o0:o1] - hh * hh)) == 0.0
        assert np.max(np.abs(W2[o0:o1] - W)) <= 1e-14 * np.max(np.abs(W)), j


@pytest.mark.parametrize("solver", ["auto", "auto_small"])
def test_mixed_plan_windows_and_two_pass_tiles(solver):
    """One context whose plan mixes both solvers: bar instances go to
    windows, while a solitary wave at lambda = 3e5 on dx = 0.01 (halo
    estimate ~1660 rows, beyond a quarter of either window width) falls
    back to the exact two-pass tiles; every instance matches the oracle.
    At lambda = 3e5 the oracle's own result moves by 5e-10 (relative) under
    a half-ulp perturbation of its input, so the state bar is max(1e-11,
    8x that sensitivity), as for every field bar."""
    Solver = _solver()
    wl = WL.concat("mixed plan", [WL.batched_bar(n_inst=6, seed=9, n_lo=600, n_hi=9000),
                                  WL.solitary(N=5000, L=50.0, lam=3e5, t_end=0.0),
                                  WL.dam_break(N=3000, xa=-45.0, xb=45.0)])
    s = Solver.from_workload(wl, solver=solver)
    info = s.plan_info()
    s.close()
    mode = info["mode"]
    assert mode[6] == 1 and (mode[:6] == 0).all(), mode
    assert info["windows"] > 0 and info["exact_tiles"] > 0
    assert (info["halo"][mode == 0] > 0).all()
    compare(wl, 50, label="mixed plan", solver=solver, state_sens=True)


def _far_from_equilibrium():
    """lambda = 1e4, dx = 0.04, N = 8000, h ~ 0.4 at rest: one instance
    starts at eta = 2 h (m = 2 h^2), one at eta = h."""
    parts = []
    for fac in (2.0, 1.0):
        n, dx = 8000, 0.04
        h = 0.4 * (1.0 + 0.01 * np.sin(2 * np.pi * np.arange(n) / n))
        part = WL._part(n, dx, 1e4, 1, h, np.zeros(n), np.zeros(n))
        part["m"] = np.ascontiguousarray(fac * h * h)
        parts.append(part)
    return WL._pack("far from equilibrium", parts, 3)


@pytest.mark.parametrize("solver", ["auto", "auto_small"])
def test_window_certificate_flags_an_insufficient_halo(solver):
    """At eta = 2 h the stage's depth rows couple far more strongly than the
    rest state the planner sizes the halo from (392 rows): from the
    oracle's own rows, about 700 rows are needed for 2^-60.  The windowed
    solve must then flag that instance (HSGN_EWINDOW, status bit 4) instead
    of returning a truncated result; the instance at eta = h is not
    flagged, and the exact solver matches the oracle on both (the state
    bar follows the oracle's own half-ulp sensitivity: 1e-10 of the state
    at eta = 2 h, where the relaxation drives W to about 12)."""
    from paper_2510_07539_amd.hsgn import HSGN_EWINDOW
    wl = _far_from_equilibrium()
    # the oracle's rows at the first stage: decay rate of the depth system
    n, prm, b, U0 = wl.instance(0)
    p = O.make_params(**prm)
    tau = (1.0 - 1.0 / np.sqrt(2.0)) * O.dt(p, U0[0], U0[1])
    rc, _, A = O.stage(p, tau, b, U0, U0, debug=True)
    assert rc == 0
    ratio = np.max((np.abs(A["lo"]) + np.abs(A["up"])) / np.abs(A["di"]))
    R = ratio / (2.0 * (1.0 - ratio))
    qq = 1.0 + 0.5 / R
    need = 60.0 * np.log(2.0) / -np.log(qq - np.sqrt(qq * qq - 1.0))
    Solver = _solver()
    s = Solver.from_workload(wl, solver=solver)
    info = s.plan_info()
    assert (info["mode"] == 0).all() and info["halo"][0] < 0.75 * need, (info["halo"], need)
    s.step(1)
    rc, flags = s.status()
    s.close()
    assert rc == HSGN_EWINDOW, rc
    assert flags[0] & 4 and not flags[1] & 4, flags
    compare(wl, 3, label="far from equilibrium, exact", solver="exact", state_sens=True)


@pytest.mark.parametrize("solver", ["auto_small", "exact"])
def test_nonphysical_instance_flagged_at_the_oracle_step(solver):
    """Instance 1469 of the batched bar (N = 566, lambda = 1e4), the first of
    the batch to fail: the oracle's step 280 produces a non-physical state.
    Run within the full batch (graph blocks of 40 steps, halo margin 1 with
    the halo retry, as the benchmark runs), the library must flag that
    instance, and no other, with the non-physical bit in step 280, and
    none before."""
    from paper_2510_07539_amd.hsgn import HSGN_ENONPHYS
    Solver = _solver()
    wl = WL.batched_bar()
    j = 1469
    n, prm, b, U0 = wl.instance(j)
    p = O.make_params(**prm)
    assert O.run(p, b, U0, 0.0, 279)[0] == 0 and O.run(p, b, U0, 0.0, 280)[0] == 1
    s = Solver.from_workload(wl, solver=solver)
    if solver == "auto_small":
        s.set_halo_margin(1.0)
        s.set_halo_retry(True)
    s.run(240, block=40)
    s.step(39)
    rc, flags = s.status()
    assert rc == 0, (rc, np.nonzero(flags))
    s.step(1)
    rc, flags = s.status()
    assert rc == HSGN_ENONPHYS and flags[j] & 1, (rc, flags[j])
    assert np.nonzero(flags)[0].tolist() == [j]
    s.close()


@pytest.mark.parametrize("solver", ["auto", "exact"])
def test_coercivity_loss_flagged_at_the_oracle_step(solver):
    """Instance 84 of the batched bar (N = 586, lambda = 1e3): its solitary
    wave steepens over the bar crest and the oracle's stage 2 of step 368
    meets beta <= 0 (min beta 49 one step earlier, -31 there: a clear
    crossing).  The library must match the oracle up to step 367, flag the
    instance non-coercive at step 368, and then keep it frozen.  One step
    before the crossing the oracle's own half-ulp sensitivity is 5.6e-11
    relative in the state (4.6e-13 at step 300), so the state bar follows it
    (bar (1) with state_sens)."""
    from paper_2510_07539_amd.hsgn import HSGN_ENONCOERCIVE
    Solver = _solver()
    wl = WL.batched_bar().subset([84], name="bar-84")
    n, prm, b, U0 = wl.instance(0)
    p = O.make_params(**prm)
    orc, _, _ = O.run(p, b, U0, 0.0, 368)
    assert orc == 2  # oracle: non-coercive at step 368 ...
    orc, _, _ = O.run(p, b, U0, 0.0, 367)
    assert orc == 0  # ... and not before
    note("coercivity loss [%s]: N=%d, 367 steps" % (solver, n))
    s = Solver.from_workload(wl, solver=solver)
    s.step(367)
    rc, flags = s.status()
    assert rc == 0 and flags[0] == 0
    (h, q, m, W), t = s.get_state()
    check_instance(0, [x.cpu().numpy() for x in (h, q, m, W)], wl, 367, state_sens=True)
    s.step(1)
    rc, flags = s.status()
    assert rc == HSGN_ENONCOERCIVE and flags[0] & 2, (rc, flags)
    (h1, q1, m1, W1), t1 = s.get_state()
    s.step(3)
    (h2, q2, m2, W2), t2 = s.get_state()
    assert float(t2[0]) == float(t1[0])
    for a, c in ((h1, h2), (q1, q2), (m1, m2), (W1, W2)):
        assert torch.equal(a, c)
    s.close()


@pytest.mark.parametrize("solver", SOLVERS)
def test_paper_test_problems(solver):
    """The paper's Gaussian bell (lambda 100 and 5000), smooth hump, Favre
    bores (eps 1.1 and 1.3) and shelf, 5000 cells each, 300 steps."""
    compare(WL.paper_tests(), 300, label="paper tests", solver=solver)


def _modes_case():
    return WL.concat("per-instance modes", [WL.batched_bar(n_inst=6, seed=9, n_lo=600, n_hi=9000),
                                           WL.solitary(N=5000, L=1250.0, lam=1000.0, t_end=0.0),
                                           WL.dam_break(N=3000, xa=-45.0, xb=45.0)])


def test_per_instance_solver_modes_match_the_oracle():
    """hsgn_set_instance_solvers: one batch with instances in each of the
    three modes (4096-row windows, 2048-row windows, the exact two-pass
    solve: two window launches and the two-pass launches in every stage)
    matches the oracle instance by instance."""
    Solver = _solver()
    wl = _modes_case()
    modes = ["auto", "auto_small", "exact", "auto_small", "auto", "exact", "auto_small", "auto"]
    s = Solver.from_workload(wl)
    s.set_instance_solvers(modes)
    info = s.plan_info()
    note("  plan: %d windows (rows %d), %d two-pass tiles" % (
        info["windows"], info["window_rows"], info["exact_tiles"]))
    assert info["window_rows"] == -1 and info["exact_tiles"] > 0
    assert [int(x) for x in info["mode"]] == [0, 0, 1, 0, 0, 1, 0, 0]
    s.step(30)
    (h, q, m, W), t = s.get_state()
    rc, _ = s.status()
    s.close()
    assert rc == 0
    U = [x.cpu().numpy() for x in (h, q, m, W)]
    for j in range(wl.n_inst):
        check_instance(j, U, wl, 30)


def _equal_states(a, b):
    (Ua, ta), (Ub, tb) = a.get_state(), b.get_state()
    for x, y in zip(Ua, Ub):
        assert torch.equal(x, y)
    assert torch.equal(ta, tb)
    return Ua


def test_persistent_launch_bitwise_equals_grid():
    """HSGN_LAUNCH_PERSISTENT computes each window exactly as the grid launch
    does: on a batch with both window widths and two-pass instances (flat
    and bed instances, both boundary types), eager steps and replays of a
    captured graph, with eager steps between them, equal the grid launch's
    bitwise; the result matches the oracle."""
    Solver = _solver()
    wl = _modes_case()
    modes = ["auto", "auto_small", "exact", "auto_small", "auto", "exact", "auto_small", "auto"]
    a = Solver.from_workload(wl)
    b = Solver.from_workload(wl)
    for s in (a, b):
        s.set_instance_solvers(modes)
    b.set_launch("persistent")
    a.step(10)
    b.step(10)
    _equal_states(a, b)
    b.run(20, block=10)
    b.step(3)
    b.run(20, block=10)
    a.step(43)
    U = _equal_states(a, b)
    for s in (a, b):
        rc, _ = s.status()
        assert rc == 0
    a.close()
    b.close()
    U = [x.cpu().numpy() for x in U]
    for j in range(wl.n_inst):
        check_instance(j, U, wl, 53)


@pytest.mark.parametrize("case", ["bar_auto", "bar_auto_small", "flat_long"])
def test_persistent_launch_full_size_bitwise(case):
    """At full size (thousands of windows: more than the resident
    workgroups, so each takes many windows from its XCD's queue and then
    from the other queues) the persistent launch equals the grid launch
    bitwise, over graph replays and eager steps: the batched workload over
    the bar in both window widths, and the 2^24-cell periodic flat run."""
    Solver = _solver()
    if case == "flat_long":
        wl, solver = WL.long_periodic(), "auto_small"
    else:
        wl, solver = WL.batched_bar(), case[4:]
    note("persistent vs grid: %s, %d cells, %s" % (case, wl.n_cells, solver))
    a = Solver.from_workload(wl, solver=solver)
    b = Solver.from_workload(wl, solver=solver)
    b.set_launch("persistent")
    note("  %d windows" % b.plan_info()["windows"])
    for s in (a, b):
        s.run(20, block=10)
        s.step(3)
        s.run(10, block=10)
    _equal_states(a, b)
    for s in (a, b):
        rc, _ = s.status()
        assert rc == 0
    a.close()
    b.close()


def test_autotune_launch_keeps_state_and_faster_launch():
    """hsgn_autotune_launch leaves the loaded state, time and status bitwise
    as they were and keeps the launch with the smaller measured time; the
    steps that follow equal the grid launch's bitwise."""
    Solver = _solver()
    wl = WL.batched_bar(n_inst=64, seed=17, n_lo=4000, n_hi=30000, nsteps=10)
    s = Solver.from_workload(wl, solver="auto_small")
    (h0, q0, m0, W0), t0 = s.get_state()
    kept, ms = s.autotune_launch(3)
    note("autotune_launch: kept %s, ms/step %s" % (kept, ms))
    assert kept == min(ms, key=ms.get)
    (h1, q1, m1, W1), t1 = s.get_state()
    for x, y in ((h0, h1), (q0, q1), (m0, m1), (W0, W1), (t0, t1)):
        assert torch.equal(x, y)
    g = Solver.from_workload(wl, solver="auto_small")
    s.step(10)
    g.step(10)
    _equal_states(s, g)
    s.close()
    g.close()


def test_autotune_classes_table_round_trip():
    """hsgn_autotune_classes: every instance is in one class, the loaded
    state is left bitwise as it was, and a context that applies the stored
    table (through JSON) gets the same plan: both step bitwise alike, and
    match the oracle."""
    import json
    Solver = _solver()
    wl = WL.concat("tuner", [WL.batched_bar(n_inst=20, seed=13, n_lo=512, n_hi=12000),
                             WL.solitary(N=800, t_end=0.0)])
    s = Solver.from_workload(wl)
    (h0, q0, m0, W0), t0 = s.get_state()
    table = s.autotune_classes(2)
    note("  kept %s; whole batch %s; %d classes" % (table["kept"], table["whole_batch_ms_per_step"],
                                                    len(table["classes"])))
    (h1, q1, m1, W1), t1 = s.get_state()
    for a, b in zip((h0, q0, m0, W0, t0), (h1, q1, m1, W1, t1)):
        assert torch.equal(a, b)
    assert sum(c["instances"] for c in table["classes"]) == wl.n_inst
    assert sum(c["cells"] for c in table["classes"]) == wl.n_cells
    keys = [tuple(sorted(c["key"].items())) for c in table["classes"]]
    assert len(set(keys)) == len(keys)
    for c in table["classes"]:
        assert c["kept"] in ("auto", "exact", "auto_small")
        assert min(c["ms_per_step"].values()) > 0
    assert table["kept"] in ("auto", "exact", "auto_small", "per_class")
    stored = json.loads(json.dumps(table))
    s2 = Solver.from_workload(wl)
    s2.apply_table(stored)
    p1, p2 = s.plan_info(), s2.plan_info()
    assert np.array_equal(p1["mode"], p2["mode"]) and p1["windows"] == p2["windows"]
    assert p1["window_rows"] == p2["window_rows"] and p1["exact_tiles"] == p2["exact_tiles"]
    s.step(20)
    s2.step(20)
    Ua, _ = s.get_state()
    Ub, _ = s2.get_state()
    for a, b in zip(Ua, Ub):
        assert torch.equal(a, b)
    U = [x.cpu().numpy() for x in Ua]
    s.close()
    s2.close()
    for j in (0, 7, 19, 20):
        check_instance(j, U, wl, 20)


def test_autotune_keeps_state_and_fastest_mode():
    """The autotuner leaves the loaded state, time and status untouched
    (bitwise), keeps the mode with the smallest measured time, and the
    solver then still matches the oracle."""
    Solver = _solver()
    wl = WL.concat("tune", [WL.batched_bar(n_inst=6, seed=9, n_lo=600, n_hi=9000, nsteps=20),
                            WL.solitary(N=3000, L=750.0, lam=1000.0, t_end=0.0, nsteps=20)],
                   nsteps=20)
    s = Solver.from_workload(wl)
    (h0, q0, m0, W0), t0 = s.get_state()
    kept, ms = s.autotune(3)
    note("autotune: kept %s, ms/step %s" % (kept, ms))
    assert kept == min(ms, key=ms.get)
    (h1, q1, m1, W1), t1 = s.get_state()
    for a, b in ((h0, h1), (q0, q1), (m0, m1), (W0, W1), (t0, t1)):
        assert torch.equal(a, b)
    rc, flags = s.status()
    assert rc == 0
    s.step(20)
    (h, q, m, W), t = s.get_state()
    U = [x.cpu().numpy() for x in (h, q, m, W)]
    for j in range(wl.n_inst):
        check_instance(j, U, wl, 20)
    s.close()


@pytest.mark.parametrize("solver", SOLVERS)
def test_first_order_scheme(solver):
    """The first-order scheme (one stage, tau = dt, no reconstruction) on a
    mix: periodic solitary waves (one tile, several windows), the bar batch,
    the dam break and the paper's shelf, 100 steps, through hsgn_run."""
    wl = WL.concat("first-order", [
        WL.solitary(N=800, lam=100.0, t_end=0.0),
        WL.solitary(N=9000, L=2250.0, lam=1000.0, t_end=0.0),
        WL.batched_bar(n_inst=4, seed=12, n_lo=700, n_hi=7000),
        WL.dam_break(N=6000, xa=-90.0, xb=90.0),
        WL.shelf()], nsteps=100)
    compare(wl, 100, use_run=True, block=20, label="first order", solver=solver, order=1)


def test_first_order_adjoint_is_rejected():
    from paper_2510_07539_amd.hsgn import HsgnError
    Solver = _solver()
    wl = WL.solitary(N=200, L=50.0, t_end=0.0)
    wl.dt_fixed[:] = 0.01
    s = Solver.from_workload(wl, order=1)
    z = torch.from_numpy(wl.h).cuda()
    with pytest.raises(HsgnError):
        s.adjoint(3, 2, torch.zeros((1, 1), dtype=torch.int32), torch.zeros((1, 3, 1)), z)
    s.close()


# ---------------------------------------------------------------------------
# Fully explicit hSGN scheme with Heun's method (Sec. 4.1, flat bottom,
# CFL 0.4 on |u| + c as in the paper's comparisons)
# ---------------------------------------------------------------------------
EXS = 1  # scheme: explicit
CFL_EX = 0.4


def _flat_mix():
    a = WL.solitary(N=800, lam=100.0, t_end=0.0)                # periodic, one tile
    b = WL.solitary(N=3001, L=750.25, lam=1000.0, t_end=0.0)    # periodic, ragged tiles
    c = WL.batched_flat(n_inst=6, seed=17, n_lo=513, n_hi=5000)  # transmissive, ragged
    return WL.concat("explicit mix", [a, b, c])


def test_explicit_parity_mix():
    compare(_flat_mix(), 60, label="explicit Heun", scheme=EXS, cfl=CFL_EX)


def test_explicit_edge_sizes():
    parts = []
    for n in (4, 5, 7, 1023, 1024, 1025, 2049):
        for bc in (0, 1):
            parts.append(WL.solitary(N=n, L=n * 0.25, lam=300.0, t_end=0.0, bc=bc))
    compare(WL.concat("explicit edge sizes", parts), 25, label="explicit sizes", scheme=EXS,
            cfl=CFL_EX)


def test_explicit_graph_replay_equals_eager_and_t_end():
    Solver = _solver()
    wl = _flat_mix()
    s1 = Solver.from_workload(wl, scheme=EXS, cfl=CFL_EX)
    s1.step(40)
    s2 = Solver.from_workload(wl, scheme=EXS, cfl=CFL_EX)
    s2.run(40, block=20)
    s2.step(1)
    s2.run(19, block=20)
    s1.step(20)
    (a, ta), (b, tb) = s1.get_state(), s2.get_state()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    assert torch.equal(ta, tb)
    s1.close()
    s2.close()
    # t_end: the last step is clamped and the instance then stays frozen
    wl = WL.solitary(N=600, L=150.0, lam=100.0, t_end=0.05)
    compare(wl, 40, label="explicit to t_end", scheme=EXS, cfl=CFL_EX)


def test_explicit_rejects_bed_adjoint_and_autotune():
    from paper_2510_07539_amd.hsgn import HsgnError
    Solver = _solver()
    with pytest.raises(HsgnError):
        Solver.from_workload(WL.batched_bar(n_inst=2, seed=1, n_lo=600, n_hi=900), scheme=EXS)
    wl = WL.solitary(N=200, L=50.0, t_end=0.0)
    wl.dt_fixed[:] = 0.001
    s = Solver.from_workload(wl, scheme=EXS)
    with pytest.raises(HsgnError):
        s.autotune()
    z = torch.from_numpy(wl.h).cuda()
    with pytest.raises(HsgnError):
        s.adjoint(3, 2, torch.zeros((1, 1), dtype=torch.int32), torch.zeros((1, 3, 1)), z)
    s.close()


def test_explicit_batched_flat_full_size_sampled():
    """The flat batched workload at its full size (4096 instances, 3.4e7
    cells), 20 steps; 16 instances spread over the batch against the oracle."""
    wl = WL.batched_flat()
    insts = list(range(0, wl.n_inst, wl.n_inst // 16))
    compare(wl, 20, use_run=True, block=10, insts=insts, label="batched flat full size",
            scheme=EXS, cfl=CFL_EX)


# ---------------------------------------------------------------------------
# Standard SGN equations, elliptic-hyperbolic form (Sec. 4.3-4.4), flat
# bottom, Heun's method, CFL 0.9 on |u| + sqrt(g h)
# ---------------------------------------------------------------------------
SGNS = 2  # scheme: standard SGN


def _sgn_mix():
    a = WL.solitary(N=800, t_end=0.0)                               # periodic, register solve
    b = WL.solitary(N=5001, L=1250.25, t_end=0.0)                   # periodic, > 4096 rows
    c = WL.batched_flat(n_inst=6, seed=19, n_lo=513, n_hi=9000)      # transmissive, mixed
    return WL.concat("sgn mix", [a, b, c])


SGN_SOLVERS = ["auto", "exact"]  # windowed phi solve where planned / two-pass everywhere


@pytest.mark.parametrize("solver", SGN_SOLVERS)
def test_sgn_parity_mix(solver):
    """The phi solve in both forms: "auto" plans windows (single pass, the
    instances longer than a window truncated at certified edges), "exact"
    the two-pass tiled solve for every instance."""
    wl = _sgn_mix()
    s = _solver().from_workload(wl, scheme=SGNS, solver=solver)
    info = s.plan_info()
    s.close()
    note("  SGN plan [%s]: %d windows, %d two-pass tiles, halo max %d" % (
        solver, info["windows"], info["exact_tiles"], int(info["halo"].max())))
    if solver == "auto":
        assert info["windows"] > wl.n_inst  # some instance spans several windows
    else:
        assert info["windows"] == 0
    compare(wl, 40, label="SGN Heun", scheme=SGNS, solver=solver)


@pytest.mark.parametrize("solver", SGN_SOLVERS)
def test_sgn_edge_sizes(solver):
    parts = []
    for n in (4, 5, 7, 1023, 1024, 1025, 4096, 4097):
        for bc in (0, 1):
            parts.append(WL.solitary(N=n, L=n * 0.25, t_end=0.0, bc=bc))
    compare(WL.concat("sgn edge sizes", parts), 20, label="SGN sizes", scheme=SGNS, solver=solver)


@pytest.mark.parametrize("scheme", [0, SGNS])
def test_halo_margin_short_halos_are_flagged(scheme):
    """hsgn_set_halo_margin: with a far too small safety factor the halos
    shrink to a few rows, and a window whose truncation then reaches its
    core must flag its instance (HSGN_EWINDOW, status bit 4) instead of
    returning a truncated result; instances solved in one window are not
    flagged; back at the default factor the same state steps without a
    flag and matches the oracle."""
    from paper_2510_07539_amd.hsgn import HSGN_EWINDOW
    Solver = _solver()
    if scheme == SGNS:
        wl = WL.batched_flat(n_inst=6, seed=19, n_lo=513, n_hi=9000)
    else:
        wl = WL.batched_bar(n_inst=6, seed=19, n_lo=513, n_hi=9000)
    s = Solver.from_workload(wl, scheme=scheme)
    full = s.plan_info()
    s.set_halo_margin(1e-4)
    info = s.plan_info()
    note("  halos at the default factor %s, at 1e-4 %s" % (list(full["halo"]), list(info["halo"])))
    assert (info["halo"] <= full["halo"]).all() and info["halo"].max() < full["halo"].max()
    single = wl.sizes() <= 4096  # one window of 4096 rows: exact, never flagged
    assert not single.all() and (info["mode"] == 0).all()
    s.step(1)
    rc, flags = s.status()
    assert rc == HSGN_EWINDOW, rc
    # an instance of two windows keeps a wide overlap whatever the halo (each
    # window covers 4096 of its rows), so it may pass; the longest, of three
    # windows with 8-row halos, must not
    longest = int(np.argmax(wl.sizes()))
    assert flags[longest] & 4, flags
    for j in range(wl.n_inst):
        if single[j]:
            assert not flags[j] & 4, (j, flags)
    s.close()
    s = Solver.from_workload(wl, scheme=scheme)
    s.set_halo_margin(2.0)
    s.step(5)
    (h, q, m, W), _ = s.get_state()
    rc, _ = s.status()
    assert rc == 0
    U = [x.cpu().numpy() for x in (h, q, m, W)]
    s.close()
    for j in range(wl.n_inst):
        check_instance(j, U, wl, 5, scheme=scheme)


@pytest.mark.parametrize("scheme", [0, SGNS])
def test_halo_retry_recovers_short_halos(scheme):
    """hsgn_set_halo_retry: at the far too small factor of the test above,
    with the retry on, a block whose windows flag is run again from a copy
    of its initial state with the flagged instances at twice their margin
    until every window certifies its truncation; the result carries no
    flag and matches the oracle, in one eager call and in graph blocks with
    an eager remainder.  Only instances that flagged grow their margin
    (those solved in one window keep 1e-4), and the grown margins are kept:
    after a reload the same steps need no retry."""
    Solver = _solver()
    if scheme == SGNS:
        wl = WL.batched_flat(n_inst=6, seed=19, n_lo=513, n_hi=9000)
    else:
        wl = WL.batched_bar(n_inst=6, seed=19, n_lo=513, n_hi=9000)
    single = wl.sizes() <= 4096  # one window: exact, never flagged
    for mode in ("step", "run"):
        s = Solver.from_workload(wl, scheme=scheme)
        s.set_halo_margin(1e-4)
        s.set_halo_retry(True)
        if mode == "step":
            s.step(5)
        else:
            s.run(5, block=2)
        rc, flags = s.status()
        assert rc == 0, (mode, rc, flags)
        margins, retries = s.halo_state()
        note("  %s: halo margins 1e-4 -> %s after %d blocks run again" % (
            mode, np.array2string(margins, precision=3), retries))
        assert retries >= 1 and margins.max() > 1e-4
        assert (margins[single] == 1e-4).all()
        (h, q, m, W), _ = s.get_state()
        U = [x.cpu().numpy() for x in (h, q, m, W)]
        for j in range(wl.n_inst):
            check_instance(j, U, wl, 5, scheme=scheme)
        # reload: the kept margins certify the same steps at once
        s.set_state(torch.from_numpy(wl.h).cuda(), torch.from_numpy(wl.q).cuda(),
                    torch.from_numpy(wl.m).cuda(), torch.from_numpy(wl.W).cuda())
        s.step(5)
        assert s.status()[0] == 0
        m2, r2 = s.halo_state()
        assert r2 == 0 and np.array_equal(m2, margins)
        # a new base margin resets the per-instance ones
        s.set_halo_margin(1.0)
        assert (s.halo_state()[0] == 1.0).all()
        s.close()


@pytest.mark.parametrize("scheme", [0, SGNS])
def test_two_runs_bitwise_identical(scheme):
    """Determinism: the same workload in two fresh contexts gives the same
    state bit for bit (no floating-point atomics: only the speed and depth
    maxima use atomics, on their bit patterns, which is order-independent),
    with windows of both widths in one batch."""
    Solver = _solver()
    if scheme == SGNS:
        wl = WL.batched_flat(n_inst=24, seed=31, n_lo=513, n_hi=12000)
    else:
        wl = WL.batched_bar(n_inst=24, seed=31, n_lo=513, n_hi=12000)
    out = []
    for _ in range(2):
        s = Solver.from_workload(wl, scheme=scheme)
        s.run(30, block=10)
        out.append(s.get_state())
        assert s.status()[0] == 0
        s.close()
    (a, ta), (b, tb) = out
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    assert torch.equal(ta, tb)


def test_sgn_graph_replay_equals_eager_and_t_end():
    Solver = _solver()
    wl = _sgn_mix()
    s1 = Solver.from_workload(wl, scheme=SGNS)
    s1.step(40)
    s2 = Solver.from_workload(wl, scheme=SGNS)
    s2.run(40, block=20)
    (a, ta), (b, tb) = s1.get_state(), s2.get_state()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    assert torch.equal(ta, tb)
    s1.close()
    s2.close()
    compare(WL.solitary(N=600, L=150.0, t_end=0.3), 40, label="SGN to t_end", scheme=SGNS)


def test_sgn_rejects_bed_adjoint_and_autotune():
    from paper_2510_07539_amd.hsgn import HsgnError
    Solver = _solver()
    with pytest.raises(HsgnError):
        Solver.from_workload(WL.batched_bar(n_inst=2, seed=1, n_lo=600, n_hi=900), scheme=SGNS)
    wl = WL.solitary(N=200, L=50.0, t_end=0.0)
    wl.dt_fixed[:] = 0.01
    s = Solver.from_workload(wl, scheme=SGNS)
    with pytest.raises(HsgnError):
        s.autotune()
    z = torch.from_numpy(wl.h).cuda()
    with pytest.raises(HsgnError):
        s.adjoint(3, 2, torch.zeros((1, 1), dtype=torch.int32), torch.zeros((1, 3, 1)), z)
    s.close()


@pytest.mark.parametrize("solver,margin", [(m, None) for m in SGN_SOLVERS] + [("auto", 1.0)])
def test_sgn_batched_flat_full_size_sampled(solver, margin):
    """The flat batch with the SGN solver at full size, in both forms of the
    phi solve at the default halo margin and at margin 1 with the halo retry
    (the benchmark's configuration); instances sampled for the oracle."""
    wl = WL.batched_flat()
    insts = list(range(0, wl.n_inst, wl.n_inst // 16))
    sizes = wl.sizes()
    insts.append(int(np.argmax(sizes)))  # the most windows
    compare(wl, 20, use_run=True, block=10, insts=sorted(set(insts)),
            label="SGN batched flat full size", scheme=SGNS, solver=solver,
            margin=margin, retry=margin is not None)


def test_dam_break_full_run():
    """C2 at its full size and length: 20000 cells, 2000 steps, graph blocks
    of 100 (the oracle runs all of it)."""
    compare(WL.dam_break(), 2000, use_run=True, block=100, label="C2 2000 steps")


GAMMA = 1.0 - 1.0 / np.sqrt(2.0)
GOLDEN_C4 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                         "c4_long_periodic_100.npz")


def seam_drift_bound(wl, n_seams, stages, hmin, hmax):
    """Bound on the momentum sum's drift of a periodic flat instance solved in
    windows: at a seam each window takes its neighbour's depth from its own
    halo row; the certificate bounds the truncation at a core edge by 2^-56
    of the depth, and one row further out by 1/rho of that (rho: decay of
    the depth system's inverse per row).  The two pressures P = S + beta h
    of the seam's cells then differ between the windows by at most
    beta h 2^-56 (1 + 1/rho) each, and the central pressure differences
    stop telescoping there: per seam and stage the sum of q moves by at most
    (tau/dx) beta_max h_max 2^-56 (1 + 1/rho).  Upper bounds over the run:
    tau from dt <= CFL dx / sqrt(g h_max), beta <= g h + 2 lambda/3; rho
    from the rest-state coefficients at the shallowest cell and the
    smallest tau, the weakest coupling."""
    g, lam, dx, cfl = float(wl.g[0]), float(wl.lam[0]), float(wl.dx[0]), float(wl.cfl[0])
    tau_max = GAMMA * cfl * dx / np.sqrt(g * hmin)
    tau_min = GAMMA * cfl * dx / (np.sqrt(g * hmax) + 1.0)  # |u| < 1 m/s here
    beta_max = g * hmax + 2.0 * lam / 3.0
    beta_min = g * hmin + (2.0 * lam / 3.0) / (1.0 + lam * tau_max ** 2 / hmin ** 2)
    R = (tau_min / dx) ** 2 * beta_min
    qq = 1.0 + 0.5 / R
    rho = qq - np.sqrt(qq * qq - 1.0)
    per = (tau_max / dx) * beta_max * hmax * 2.0 ** -56 * (1.0 + 1.0 / rho)
    return stages * n_seams * per


def test_long_periodic_full_size_properties():
    """C4 at its full size (2^24 cells, 200 steps): mass and momentum
    conservation (periodic, flat bed) in every solver mode, and the windowed
    solves against the exact two-pass solve.

    Momentum: with the exact solver the central pressure differences and
    the Rusanov fluxes telescope, so the sum of q moves by rounding only:
    |d sum q| <= 1e-13 sum|q|.  The windowed solves conserve it only up to
    the certified truncation at their window seams (seam_drift_bound); the
    seam count is the plan's window count.  Mass: relative 1e-12 (observed
    1e-13).

    Windowed vs exact: the bars of the oracle comparison, with the
    sensitivity measured on the library itself (a third run from the state
    perturbed by 2^-53 relative): at lambda = 1e4 the stiff field W moves
    by about 1e-11 of the state under such a perturbation."""
    Solver = _solver()
    wl = WL.long_periodic()
    note("C4 full: %d cells, 200 steps" % wl.n_cells)
    res = {}
    rng = np.random.default_rng(0)
    sign = torch.from_numpy(rng.choice([-1.0, 1.0], size=wl.n_cells)).cuda()
    for solver in ("exact", "auto", "auto_small", "perturbed"):
        s = Solver.from_workload(wl, solver="auto" if solver == "perturbed" else solver)
        nwin = s.plan_info()["windows"]
        (h0, q0, m0_, W0), _ = s.get_state()
        if solver == "perturbed":
            f = 1.0 + 2.0 ** -53 * sign
            s.set_state(h0 * f, q0 * f, m0_ * f, W0 * f)
            (h0, q0, _, _), _ = s.get_state()
        m0, p0 = float(h0.sum()), float(q0.sum())
        s.run(200, block=100)
        rc, flags = s.status()
        assert rc == 0, (solver, rc)
        (h, q, m, W), t = s.get_state()
        mass, mom = float(h.sum()), float(q.sum())
        absq = float(q.abs().sum())
        hmin = min(float(h0.min()), float(h.min()))
        hmax = max(float(h0.max()), float(h.max()))
        bound = 1e-13 * absq
        if nwin > 0:
            bound += seam_drift_bound(wl, nwin, 400, hmin, hmax)
        note("  %s: %d windows, mass drift %.2e, momentum drift %.2e (bound %.2e, sum |q| %.3e)"
             % (solver, nwin, abs(mass - m0) / m0, abs(mom - p0), bound, absq))
        assert abs(mass - m0) <= 1e-12 * m0
        assert abs(mom - p0) <= bound, (solver, abs(mom - p0), bound)
        if solver == "exact":
            assert nwin == 0
        res[solver] = (h, q, m, W)
        s.close()
    scale = max(float(x.abs().max()) for x in res["exact"])
    sens = [float((a - b).abs().max()) for a, b in zip(res["auto"], res["perturbed"])]
    for solver in ("auto", "auto_small"):
        dev = [float((a - b).abs().max()) for a, b in zip(res[solver], res["exact"])]
        note("  %s vs exact per field %s; sensitivity %s" % (
            solver, ["%.1e" % d for d in dev], ["%.1e" % d for d in sens]))
        assert max(dev) / scale <= max(1e-11, 8.0 * max(sens) / scale)
        for fld in range(4):
            fmax = float(res["exact"][fld].abs().max())
            assert dev[fld] <= max(1e-11 * fmax, 8.0 * sens[fld], 1e-300), ("hqmW"[fld], dev, sens)


@pytest.mark.parametrize("solver,margin", [(m, None) for m in SOLVERS] + [("auto_small", 1.0)])
def test_long_periodic_full_size_vs_stored_oracle(solver, margin):
    """C4 at its full size (2^24 cells) after 100 graph-captured steps
    against the oracle's values stored by tests/golden/make_c4_golden.py
    (4096 seeded cells plus both ends of the ring): the state bar (relative
    to the oracle's maxima over all cells) and the per-field bars with the
    oracle's own half-ulp sensitivity at the same cells; the time reached;
    the sum of h against the oracle's.  In the three solver modes at the
    default halo margin, and at margin 1 with the halo retry (the
    benchmark's configuration)."""
    d = np.load(GOLDEN_C4)
    nsteps = int(d["nsteps"])
    Solver = _solver()
    wl = WL.long_periodic()
    note("C4 full vs stored oracle [%s]: %d cells, %d steps, %d sampled cells" % (
        solver, wl.n_cells, nsteps, len(d["idx"])))
    s = Solver.from_workload(wl, solver=solver)
    if margin is not None:
        s.set_halo_margin(margin)
        s.set_halo_retry(True)
    s.run(nsteps, block=100)
    rc, _ = s.status()
    assert rc == 0, rc
    (h, q, m, W), t = s.get_state()
    s.close()
    idx = torch.from_numpy(d["idx"]).cuda()
    U = np.stack([x[idx].cpu().numpy() for x in (h, q, m, W)])
    Uo, Up, umax = d["U"], d["U_perturbed"], d["umax"]
    dev = np.max(np.abs(U - Uo), axis=1)
    sens = np.max(np.abs(Up - Uo), axis=1)
    note("  deviation per field %s; oracle sensitivity %s" % (
        ["%.1e" % x for x in dev], ["%.1e" % x for x in sens]))
    assert np.max(dev) / np.max(umax) <= TOL, (dev, umax)
    for f in range(4):
        assert dev[f] <= max(TOL * umax[f], 8.0 * sens[f], 1e-300), ("hqmW"[f], dev, sens)
    tg = float(t.cpu()[0])
    assert abs(tg - float(d["t"])) <= 1e-12 * float(d["t"]), (tg, float(d["t"]))
    mass = float(h.sum())
    assert abs(mass - float(d["sums"][2])) <= 1e-12 * abs(float(d["sums"][2]))
