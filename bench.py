"""Benchmark of the gfx950 hSGN IMEX step.

Default workload: the batched ensemble -- 4096 independent 1D instances,
N_j ~ U{512..16384} cells, solitary waves over a trapezoidal bar, lambda_j
from {100, 1000, 10000}, FP64, HIP-graph-captured step blocks.  One "step" is
one full two-stage IMEX step of every instance.  Metric: cell-stage updates
per second (one cell advanced through one IMEX stage).

Prints ONE JSON line.  Also reported: the same kernels on one instance per
context with eager launches (the per-instance GPU path), the roofline of the
dominant kernel from HIP events on the library's stream, and the CPU oracle
on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E
# HBM traffic of the dominant kernels measured with rocprofv3 --pmc (FETCH_SIZE
# and WRITE_SIZE in separate runs, `bench.py --probe [--solver auto_small |
# --scheme explicit | --scheme sgn] [--halo-margin 2]`), scaled by the same
# counters on a plain 512 MiB copy (FETCH_SIZE x 1.9998, WRITE_SIZE x 1.0), in
# bytes per launch (the SGN solve: per stage, every kernel of the phi solve).
# Each entry is keyed by the workload, solver mode or scheme, halo margin, and
# the hash of the code of its kernels' sources (comments and blank lines left
# out), and reported as null once that code changes.
TRAFFIC = [
    {"kernel": "win2", "workload": "batched_bar", "solver": "auto_small", "halo_margin": 2.0,
     "sources": ["hsgn_kernels.hpp", "hsgn_window.hpp"], "hash": "fc5a69c89a42cee0",
     "fetch_bytes": 2461858717, "write_bytes": 1136103467, "bytes_per_launch": 3597962184},
    {"kernel": "win2", "workload": "batched_bar", "solver": "auto_small", "halo_margin": 1.0,
     "sources": ["hsgn_kernels.hpp", "hsgn_window.hpp"], "hash": "fc5a69c89a42cee0",
     "fetch_bytes": 2461760411, "write_bytes": 1135767947, "bytes_per_launch": 3597528358},
    {"kernel": "ex2", "workload": "batched_flat", "scheme": "explicit",
     "sources": ["hsgn_kernels.hpp", "hsgn_explicit.hpp"], "hash": "2e6dc71f10ea1fd9",
     "fetch_bytes": 2232887832, "write_bytes": 1118343168, "bytes_per_launch": 3351231000},
    {"kernel": "sgn_solve", "workload": "batched_flat", "scheme": "sgn", "halo_margin": 2.0,
     "sources": ["hsgn_kernels.hpp", "hsgn_window.hpp", "hsgn_adjoint.hpp",
                 "hsgn_explicit.hpp", "hsgn_sgn.hpp"], "hash": "dc84e81a93859e7f",
     "fetch_bytes": 676293257, "write_bytes": 273330187, "bytes_per_launch": 949623443},
    {"kernel": "sgn_solve", "workload": "batched_flat", "scheme": "sgn", "halo_margin": 1.0,
     "sources": ["hsgn_kernels.hpp", "hsgn_window.hpp", "hsgn_adjoint.hpp",
                 "hsgn_explicit.hpp", "hsgn_sgn.hpp"], "hash": "dc84e81a93859e7f",
     "fetch_bytes": 646732591, "write_bytes": 273320485, "bytes_per_launch": 920053076},
]

def src_hash(sources):
    """Hash of the kernels' sources without their comments and blank lines
    (an edit of a comment leaves the measured kernels as they were)."""
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2510_07539_amd", "csrc", f)) as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def bytes_per_cell(kind, bed):
    """Algorithmic HBM bytes per cell for one launch of a kernel kind:
    what the kernel must read and write at least once (FP64)."""
    b = 1 if bed else 0
    return {"stage1": (4 + b + 4) * 8,      # reads U^n (+ b), writes U^(1)
            "stage2": (8 + b + 4) * 8,      # reads U^n, U^(1) (+ b), writes U^{n+1}
            "win1": (4 + b + 4) * 8,
            "win2": (8 + b + 4) * 8,
            "reduce1": (4 + b) * 8,         # reads U^n (+ b)
            "reduce2": (8 + b) * 8,         # reads U^n, U^(1) (+ b)
            "ex1": (4 + 4) * 8,             # explicit Heun stage 1: reads U^n, writes U1
            "ex2": (8 + 4) * 8,             # stage 2: reads U^n and U1, writes U^{n+1}
            "sgn_solve": (2 + 1) * 8,       # SGN: reads h, q (rows formed in the solve), writes phi
            "sgn_update": (2 + 1 + 2) * 8,  # reads h, q, phi; writes h, q (stage 1)
            }.get(kind, 0)


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Bandwidth of a plain device-to-device copy of nbytes (read + write
    counted), timed with events on torch's stream: the measured ceiling the
    roofline is also reported against."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def make_workload(name):
    from paper_2510_07539_amd import workloads as WL
    if name == "batched_bar":
        return WL.batched_bar(), ("batched_bar: 4096 instances, N_j~U{512..16384} (seed 3), "
                                  "dx=0.04 m, h0=0.4 m, soliton a_j~U[0.05,0.4]h0 over a "
                                  "trapezoidal bar (0.3 m, 1:20 / 2 m crest / 1:10), "
                                  "lambda_j in {100,1000,10000}, transmissive, CFL 0.9")
    if name == "batched_flat":
        return WL.batched_flat(), ("batched_flat: the batched_bar draws on a flat bottom (4096 "
                                   "instances, N_j~U{512..16384}, seed 3, dx=0.04 m, h0=0.4 m, "
                                   "lambda_j in {100,1000,10000}), transmissive")
    if name == "dam_break":
        return WL.dam_break(), "dam_break: N=20000 on [-300,300] m, lambda=1000, transmissive"
    if name == "long_periodic":
        return WL.long_periodic(), "long_periodic: N=2^24, dx=0.01 m, lambda=1e4, periodic"
    if name == "solitary":
        w = WL.solitary(t_end=0.0)
        return w, "solitary: N=800 on [0,200] m, h0=1, a=0.2, lambda=100, periodic"
    if name == "paper_tests":
        return WL.paper_tests(), ("paper_tests: Gaussian bell (lambda 100, 5000), smooth hump, "
                                  "Favre bores (eps 1.1, 1.3), shelf; 5000 cells each")
    raise SystemExit("unknown workload " + name)


def per_instance_rate(wl, n_sample, steps, order=2, halo_margin=2.0):
    """Same kernels, one context per instance, eager launches in a host loop
    (at the batched run's halo margin; no halo retry, whose status read
    after every call would serialise the host loop)."""
    import numpy as np
    import torch
    from paper_2510_07539_amd.hsgn import Solver
    idx = np.linspace(0, wl.n_inst - 1, n_sample).astype(int)
    solvers = [Solver.from_workload(wl.subset([int(j)]), order=order) for j in idx]
    for s in solvers:
        s.set_halo_margin(halo_margin)
        s.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for s in solvers:
            s.step(1)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    cells = int(sum(wl.sizes()[idx]))
    for s in solvers:
        s.close()
    return float(order) * cells * steps / el, el, n_sample


def cpu_model():
    """Model name of the host CPU (first processor in /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, budget_s=15.0, n_sample=1024, max_steps=200, order=2):
    """The oracle (OpenMP over instances, all host threads) on a bounded
    sample: the first n_sample instances, in chunks of 5 steps until the time
    budget is spent or max_steps are done (in step 280 an instance of the
    batched bar becomes non-physical, so the sample stays in the range the
    benchmark times).  The value is the median of the chunks'
    rates; the mean over the whole sample is reported beside it."""
    import numpy as np
    import oracle as O
    sub = wl.subset(range(min(n_sample, wl.n_inst)))
    plist = [O.make_params(**sub.instance(j)[1], order=order) for j in range(sub.n_inst)]
    U = sub.state()
    t = [0.0] * sub.n_inst
    steps, el = 0, 0.0
    chunk = 5
    rates = []
    while el < budget_s and steps < max_steps:
        t0 = time.perf_counter()
        rc, U, t, st = O.run_batch(sub.offsets, plist, sub.b, U, t, chunk, nthreads=0)
        dt = time.perf_counter() - t0
        el += dt
        steps += chunk
        rates.append(float(order) * sub.n_cells * chunk / dt)
        if rc != 0:
            break
    cores = min(O.max_threads(), sub.n_inst)
    return {"value": float(np.median(rates)), "unit": "cell-stage updates/s", "cores": cores,
            "kind": "oracle", "mean": float(order) * sub.n_cells * steps / el,
            "runs": len(rates), "cpu_model": cpu_model(),
            "compiler": "gcc " + " ".join(O.COMPILE_FLAGS),
            "sample": "first %d instances (%d cells) of the same workload, %d IMEX steps in "
                      "%d runs of %d steps, %.1f s; value = median run" %
                      (sub.n_inst, sub.n_cells, steps, len(rates), chunk, el)}


def scheme_comparison(si_steps=20, halo_margin=2.0, halo_retry=False):
    """The paper's cost comparison on MI355X: the semi-implicit step (CFL 0.9
    on |u| + sqrt(g h)) against the explicit Heun step (CFL 0.4 on |u| + c)
    and the standard SGN solver (Heun, CFL 0.9), all advancing the flat
    batch to the same physical time T, one lambda at a time (the SGN run
    does not depend on lambda).  T = si_steps * 0.9 dx / max(|u| + sqrt(g h)) of the initial
    state; each run stops once every instance has reached T (t_end clamp).
    The windowed schemes run at the given halo margin and retry setting."""
    import numpy as np
    import torch
    from paper_2510_07539_amd import workloads as WL
    from paper_2510_07539_amd.hsgn import SCHEME_EXPLICIT, SCHEME_SEMI_IMPLICIT, SCHEME_SGN, Solver
    wl = WL.batched_flat()
    out = []
    for lam in (100.0, 1000.0, 10000.0):
        sub = wl.subset([j for j in range(wl.n_inst) if wl.lam[j] == lam])
        smax = float(np.max(np.abs(sub.q / sub.h) + np.sqrt(9.81 * sub.h)))
        T = si_steps * 0.9 * float(sub.dx[0]) / smax
        sub.t_end[:] = T
        row = {"lambda": lam, "instances": sub.n_inst, "cells": sub.n_cells, "T_s": T}
        for name, scheme, cfl in (("semi_implicit", SCHEME_SEMI_IMPLICIT, 0.9),
                                  ("explicit", SCHEME_EXPLICIT, 0.4),
                                  ("sgn", SCHEME_SGN, 0.9)):
            s = Solver.from_workload(sub, solver="auto_small" if scheme == 0 else None,
                                     scheme=scheme, cfl=cfl)
            if scheme != SCHEME_EXPLICIT:
                s.set_halo_margin(halo_margin)
                s.set_halo_retry(halo_retry)
            try:
                def to_T():
                    steps = 0
                    while True:
                        s.run(10, block=10)
                        steps += 10
                        _, t = s.get_state()
                        if bool((t >= T * (1 - 1e-12)).all()):
                            return steps
                # one untimed pass (code loading, graph capture), then the same
                # run again from the initial state with the cached graph
                to_T()
                s.set_state(*[torch.from_numpy(a).cuda() for a in sub.state()])
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                steps = to_T()
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                rc, _ = s.status()
            finally:
                s.close()
            row[name] = {"cfl": cfl, "steps": steps, "ms": round(1e3 * el, 2), "rc": rc}
        row["explicit_over_semi_implicit"] = round(row["explicit"]["ms"] / row["semi_implicit"]["ms"], 3)
        row["sgn_over_semi_implicit"] = round(row["sgn"]["ms"] / row["semi_implicit"]["ms"], 3)
        out.append(row)
    return out


def adjoint_cost(reps=2):
    """Cost of the gradient of the gauge misfit against the forward pass on
    the gradient workload: 1024 instances x 4096 cells over a bar plus a
    sinusoid, lambda = 1000, 200 steps, checkpoints every 20 steps.  Targets
    are the library's own gauge series from a perturbed initial surface
    (made before timing).  Forward = the loss alone (200 steps and the gauge
    misfit); adjoint = loss and both gradients (forward with checkpoints and
    tapes, the recompute of segments whose tapes did not fit, reverse
    sweep)."""
    import torch
    from paper_2510_07539_amd import workloads as WL
    from paper_2510_07539_amd.hsgn import Solver
    case = WL.adjoint_bar()
    wl, nsteps, K = case.wl, case.nsteps, case.K
    dev = "cuda"
    free_before = torch.cuda.mem_get_info()[0]
    s = Solver.from_workload(wl)
    try:
        bt = torch.from_numpy(wl.b).to(dev)
        h = torch.from_numpy(case.zeta_target).to(dev) - bt
        s.set_state(h, torch.zeros_like(h), h * h, torch.zeros_like(h))
        gi = (torch.from_numpy(wl.offsets[:-1]).to(dev)[:, None]
              + torch.from_numpy(case.gauges).to(dev).long())
        tg = torch.empty((wl.n_inst, nsteps, case.gauges.shape[1]), dtype=torch.float64, device=dev)
        for st in range(nsteps):
            s.step(1)
            (hs, _, _, _), _ = s.get_state()
            tg[:, st, :] = hs[gi]
        z = torch.from_numpy(case.zeta0).to(dev)
        g = torch.from_numpy(case.gauges).to(dev)
        s.adjoint(nsteps, K, g, tg, z, grad=True)  # allocates the workspace
        torch.cuda.synchronize()
        t_fwd, t_adj = [], []
        for _ in range(reps):
            t0 = time.perf_counter()
            s.adjoint(nsteps, K, g, tg, z, grad=False)
            torch.cuda.synchronize()
            t_fwd.append(time.perf_counter() - t0)
            t0 = time.perf_counter()
            s.adjoint(nsteps, K, g, tg, z, grad=True)
            torch.cuda.synchronize()
            t_adj.append(time.perf_counter() - t0)
    finally:
        s.close()
    f, a = min(t_fwd), min(t_adj)
    return {"workload": "adjoint_bar: 1024 instances x N=4096, dx=0.04 m, h0=0.4 m, bar (toe "
                        "~U[0.4,0.5]L) + 0.02 sin(2 pi k x/L + phi), lambda=1000, 200 steps, "
                        "K=20, 8 gauges, transmissive (seed 5, targets seed 55)",
            "forward_ms": round(1e3 * f, 2), "adjoint_ms": round(1e3 * a, 2),
            "cost_ratio": round(a / f, 3),
            "forward_cell_stages_per_s": 2.0 * wl.n_cells * nsteps / f,
            "tapes": "every segment taped in the forward pass when all tapes fit half the "
                     "free device memory (else the last two; the rest recomputed)",
            "tape_gb_all_segments": round(8.0 * nsteps * wl.n_cells * 8 / 1e9, 2),
            "device_free_gb_before": round(free_before / 1e9, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--block", type=int, default=100)
    ap.add_argument("--workload", default="batched_bar")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-per-instance", action="store_true")
    ap.add_argument("--timed-steps", type=int, default=10)
    ap.add_argument("--legs", type=int, default=5,
                    help="timed legs of --steps steps each; the value is their median")
    ap.add_argument("--solver", default="tune", choices=["tune", "auto", "exact", "auto_small"],
                    help="tune: the library times every mode on the workload and keeps the fastest")
    ap.add_argument("--launch", default="tune", choices=["tune", "grid", "persistent"],
                    help="window-stage launch; tune: the library times both and keeps the faster")
    ap.add_argument("--halo-margin", type=float, default=1.0,
                    help="safety factor of the windowed solves' halo estimates (the "
                         "library's default is 2)")
    ap.add_argument("--no-halo-retry", dest="halo_retry", action="store_false",
                    help="no halo retry (on by default: a block whose windows flag runs "
                         "again from its initial state with twice the margin)")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--table-out", default=None,
                    help="write the autotuner's table (JSON) to this file")
    ap.add_argument("--table-in", default=None,
                    help="apply a stored autotuner table (JSON) instead of tuning")
    ap.add_argument("--order", type=int, default=2, choices=[1, 2],
                    help="2: the two-stage IMEX step; 1: the first-order scheme (one stage)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the gradient workload (one timed adjoint), one JSON line")
    ap.add_argument("--probe", action="store_true",
                    help="counter probe: a plain copy of known size, then eager steps")
    ap.add_argument("--scheme", default="si", choices=["si", "explicit", "sgn"],
                    help="explicit: the fully explicit Heun step (flat batch, CFL 0.4); "
                         "sgn: the standard SGN solver (flat batch, CFL 0.9)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the semi-implicit vs explicit time-to-T comparison")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path in this library "
              "(the instances are independent, so a batch would shard across GPUs by "
              "instance with no communication).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2510_07539_amd.hsgn import Solver

    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_cost(reps=1)}))
        return
    explicit = args.scheme != "si"  # the explicit hSGN or the SGN Heun step
    if explicit and args.workload == "batched_bar":
        args.workload = "batched_flat"  # these schemes have no bed
    wl, desc = make_workload(args.workload)
    bed = wl.b is not None
    if explicit:
        from paper_2510_07539_amd.hsgn import SCHEME_EXPLICIT, SCHEME_SGN
        if args.scheme == "explicit":
            s = Solver.from_workload(wl, scheme=SCHEME_EXPLICIT, cfl=0.4)
            desc += "; explicit Heun step, CFL 0.4 on |u| + c"
        else:
            s = Solver.from_workload(wl, scheme=SCHEME_SGN)
            desc += "; standard SGN, Heun step, CFL 0.9 on |u| + sqrt(g h)"
        args.order = 2  # two Heun stages per step
    else:
        s = Solver.from_workload(wl, solver=None if args.solver == "tune" else args.solver,
                                 order=args.order)
    if args.scheme != "explicit":  # the explicit scheme has no windows
        s.set_halo_margin(args.halo_margin)
        if args.halo_retry:
            s.set_halo_retry(True)
    tuned = None
    if args.table_in and not explicit:
        # a stored autotuner table: each instance takes its class's mode
        with open(args.table_in) as fh:
            tuned = json.load(fh)
        s.apply_table(tuned)
        tuned = dict(tuned, source=os.path.basename(args.table_in))
    elif args.solver == "tune" and not args.probe and not explicit:
        # the library's tuner: a mode per class of instances (N bucket,
        # boundary, bed, halo bucket), then that plan against the three
        # uniform modes on the whole batch
        tuned = s.autotune_classes(4)
        if args.table_out:
            with open(args.table_out, "w") as fh:
                json.dump(tuned, fh, indent=1)
    launch, launch_ms = "grid", None
    if not explicit:
        if args.launch == "tune" and not args.probe:
            launch, launch_ms = s.autotune_launch(4)
            launch_ms = {k: round(v, 4) for k, v in launch_ms.items()}
        elif args.launch != "tune":
            launch = args.launch
            s.set_launch(launch)
    plan = s.plan_info()

    if args.probe:
        a = torch.empty(64 << 20, dtype=torch.float64, device="cuda")  # 512 MiB
        a.fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        s.step(3)
        torch.cuda.synchronize()
        print(json.dumps({"probe": True, "copy_bytes": a.numel() * 8, "cells": wl.n_cells}))
        return

    # Every timed leg starts from the initial state (reloaded untimed; the
    # reload also restarts the buffer rotation, so the captured graph is the
    # one replayed).  Graph blocks hold at most the timed steps (even: the
    # rotation repeats every two steps), so the timed steps replay a graph;
    # fewer than two timed steps run eagerly.
    init_state = [torch.from_numpy(a).cuda() for a in wl.state()]
    block = min(args.block, args.steps) & ~1
    s.run(args.warmup, block=max(block, 2))
    graph_warm = 0
    if block >= 2:  # capture the graph outside the timed legs (its steps run untimed)
        s.set_state(*init_state)
        s.run(block, block=block)
        graph_warm = block
    legs = []
    leg_retries = []
    for _ in range(max(args.legs, 1)):
        s.set_state(*init_state)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if block >= 2:
            s.run(args.steps, block=block)
        else:
            s.step(args.steps)
        torch.cuda.synchronize()
        legs.append(time.perf_counter() - t0)
        leg_retries.append(s.halo_state()[1])
    el = float(np.median(legs))
    rc, flags = s.status()
    if rc != 0:
        print("solver flagged %d instances" % int((flags != 0).sum()), file=sys.stderr)
        sys.exit(1)
    cell_stages = float(args.order) * wl.n_cells * args.steps  # stages per step = order
    value = cell_stages / el
    ms_step = 1e3 * el / args.steps

    # per-kernel durations from HIP events on the library's stream
    s.set_state(*init_state)
    kt = s.step_timed(args.timed_steps)
    sizes = wl.sizes()
    mode = plan["mode"]
    ex_cells = int(sizes[mode == 1].sum())
    ex_multi_cells = int(sizes[(mode == 1) & (sizes > 2048)].sum())
    win_cells = int(sizes[mode == 0].sum())
    tot = {k: v[0] for k, v in kt.items()}
    dom = max(tot, key=lambda k: tot[k])
    ms_avg, launches = kt[dom][0] / max(kt[dom][1], 1), kt[dom][1]
    cells_launch = {"reduce1": ex_multi_cells, "reduce2": ex_multi_cells, "stage1": ex_cells,
                    "stage2": ex_cells, "win1": win_cells, "win2": win_cells,
                    "ex1": wl.n_cells, "ex2": wl.n_cells,
                    "sgn_solve": wl.n_cells, "sgn_update": wl.n_cells}.get(dom, 0)
    alg_bytes = bytes_per_cell(dom, bed) * cells_launch
    achieved = alg_bytes / (ms_avg * 1e-3) / 1e9 if ms_avg > 0 else 0.0
    traffic = None
    solver_used = tuned["kept"] if tuned else args.solver
    for tr in TRAFFIC:
        if (tr["kernel"] == dom and tr["workload"] == args.workload and
                tr.get("solver", solver_used) == solver_used and
                tr.get("scheme", args.scheme) == args.scheme and
                tr.get("launch", "grid") == launch and
                tr.get("halo_margin", args.halo_margin) == args.halo_margin and
                src_hash(tr["sources"]) == tr["hash"]):
            traffic = tr["bytes_per_launch"]
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
            "kernel": (("k_win_persist<%s>" if launch == "persistent" else "k_win<%s>")
                       if dom.startswith("win") else
                       "k_ex<%s>" if dom.startswith("ex") else
                       "k_%s" if dom.startswith("sgn") else "k_stage<%s>") % dom,
            "avg_launch_ms": round(ms_avg, 4),
            "alg_bytes_per_launch": alg_bytes,
            "alg_bytes_per_cell": bytes_per_cell(dom, bed)}
    copy_gbps = copy_bandwidth()
    roof["copy_gbps"] = round(copy_gbps, 1)
    roof["frac_of_copy"] = round(achieved / copy_gbps, 4)
    step_bytes = (bytes_per_cell("stage1", bed) if args.order == 1 else
                  (bytes_per_cell("stage1", bed) + bytes_per_cell("stage2", bed)) / 2.0)
    if args.scheme == "explicit":
        step_bytes = (bytes_per_cell("ex1", False) + bytes_per_cell("ex2", False)) / 2.0
    elif args.scheme == "sgn":  # the minimum of a Heun stage: read 2 (stage 2: 4), write 2
        step_bytes = (4 + 6) / 2.0 * 8
    out = {
        "metric": "cell-stage updates/s (FP64, batched vs per-instance) at 1e-11 oracle match",
        "value": value,
        "unit": "cell-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "n_inst": wl.n_inst, "cells": wl.n_cells,
                   "graph_block_steps": block if block >= 2 else None,
                   "timed_legs_ms_per_step": [round(1e3 * x / args.steps, 4) for x in legs],
                   "graph_warmup_steps": graph_warm, "order": args.order, "scheme": args.scheme,
                   "solver": tuned["kept"] if tuned else args.solver, "autotune": tuned,
                   "window_launches": plan["window_launches"],
                   "launch": launch, "launch_ms_per_step": launch_ms,
                   "halo_margin": None if args.scheme == "explicit" else args.halo_margin,
                   "halo_retry": bool(args.halo_retry) and args.scheme != "explicit",
                   "halo_margin_max_final": (None if args.scheme == "explicit"
                                             else float(s.halo_state()[0].max())),
                   "timed_legs_blocks_run_again": leg_retries,
                   "windows": plan["windows"], "window_rows": plan["window_rows"],
                   "two_pass_tiles": plan["exact_tiles"]},
        "roofline": roof,
        "step_hbm_frac": round(value * step_bytes / 1e9 / HBM_PEAK_GBPS, 4),
        "kernel_ms_per_step": {k: round(v[0] / args.timed_steps, 4) for k, v in kt.items() if v[1]},
    }
    if not args.no_per_instance and wl.n_inst > 1 and not explicit:
        r, pel, ns = per_instance_rate(wl, 32, 3, order=args.order, halo_margin=args.halo_margin)
        out["per_instance"] = {"value": r, "unit": "cell-stage updates/s",
                               "sample": "%d instances spread over the batch, one context each, "
                                         "eager launches, 3 steps, halo margin %g without "
                                         "retry" % (ns, args.halo_margin)}
        out["batched_over_per_instance"] = value / r
    s.close()
    if not args.no_adjoint and args.workload == "batched_bar" and args.order == 2:
        out["adjoint"] = adjoint_cost()
    if not args.no_compare and args.workload == "batched_bar" and args.order == 2:
        out["scheme_comparison"] = scheme_comparison(halo_margin=args.halo_margin,
                                                     halo_retry=args.halo_retry)
    if not args.no_cpu and not explicit:
        out["cpu_baseline"] = cpu_baseline(wl, order=args.order)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
