#!/usr/bin/env python3
"""Benchmark of the self-gravity Poisson hot path on one MI355X.

Default line (the largest single-GPU workload): 512^3 intervals on the unit
box (511^3 unknowns), density of 64 seeded Gaussian clumps plus a 5%
lognormal |k|^-2 turbulent floor, 19-point sixth-order star with three ghost
layers, open boundary from the multipole expansion with lmax = 8, all-FP64
geometric multigrid V(2,2) with four-colour Gauss-Seidel, full weighting,
trilinear prolongation and an exact 7^3 coarsest solve.  One step = one whole
poisson_solve from a cold start (phi = 0): multipole boundary + V-cycles until
the relative residual is <= 1e-8.  value = unknowns x V-cycles / wall time per
step (Gcell-updates/s of the whole job, multipole included).

Beside it on the same line: the FP32 multigrid inside FP64 iterative
refinement on the same input (time and speedup), the event-timed 7-point FP64
colour pass at 511^3, the 255^3 clump workload (FP64 and mixed) and the
19-point workload at 255^3 with their errors against the CPU oracle's exact
discrete solution, a short serving leg (p50 / p99 latency and solves/s), and
the oracle timed on the host cores.  The roofline entry times the dominant
kernel (the fine-level four-colour pass) with HIP events on the plan's stream
in its solver launch configuration.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0   # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--n", type=int, default=0, help="intervals per axis (default: 512 for c3, 256 for c2)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget-s", type=float, default=12.0,
                    help="seconds of oracle V-cycles for the CPU baseline (at least one cycle)")
    ap.add_argument("--cpu-multipole", action="store_true",
                    help="also time the oracle's multipole boundary (about 25 s at 255^3)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--kernels-only", action="store_true",
                    help="for hardware-counter runs: one solve to populate the arrays, then "
                         "--sweeps resident smoother sweeps and one 1 GiB reference copy; "
                         "prints no bench line")
    ap.add_argument("--sweeps", type=int, default=10)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4", "serving", "spai"],
                    help="c3: the 511^3 19-point FP64 multigrid solve (default bench line); c2: the 255^3 "
                         "7-point one; serving: the continuous-batching request stream (its own JSON line)")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests of the serving leg on the default line")
    ap.add_argument("--no-oracle-errors", action="store_true",
                    help="skip the oracle's exact solves (errors of the 255^3 solves)")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--load", type=float, default=0.7, help="offered load relative to saturation")
    ap.add_argument("--slots", type=int, default=8, help="concurrent request slots of the full configuration")
    return ap.parse_args()


def _pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    i = min(len(xs) - 1, max(0, int(math.ceil(q / 100.0 * len(xs))) - 1))
    return xs[i]


def _time_solves(plan, rho, phi, tol, steps, warmup):
    import torch
    res = None
    for _ in range(warmup):
        phi.zero_()
        res = plan.solve(rho, phi, tol=tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        phi.zero_()
        res = plan.solve(rho, phi, tol=tol)
        if not res.converged:
            raise RuntimeError(f"solve did not converge: {res}")
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, res


def bench_c1(args):
    """32^3 cells, uniform sphere of radius 0.25 (rho = 1), multipole
    boundary with lmax 4, red-black SOR at omega_opt (and with the Chebyshev
    sequence), CG and CG preconditioned by symmetric red-black Gauss-Seidel
    to 1e-10; errors against the analytic potential and the oracle's exact
    discrete solution.  Beside it, CG against PCG on the 255^3 clump field
    (7-point) to 1e-8."""
    import torch

    import paper_2605_03563_amd as pg
    import workloads as W
    from oracle import analytic as OA
    from oracle import direct as OD
    from oracle import multipole as OM

    dev = "cuda:0"
    n, lmax, tol = 32, 4, 1e-10
    wl = W.config_c1(n=n, device=dev)
    rho = wl.rho.contiguous()
    rho_h = rho.cpu().numpy()
    ghost, _ = OM.cart_boundary(rho_h, n, 1, lmax)
    exact = OD.solve_cart(ghost, rho_h, n, 1.0 / n, 2, 1)
    x = OM.cart_coords(n, 1)[1:n]
    zz, yy, xx = np.meshgrid(x, x, x, indexing="ij")
    ana = OA.uniform_sphere(np.stack([xx, yy, zz], -1), (0.5, 0.5, 0.5), 0.25)
    s = slice(1, n)
    rows = []
    for name, method, kw in (("sor_omega_opt", "sor", {}), ("sor_chebyshev", "sor", {"omega_mode": pg.OMEGA_CHEBYSHEV}),
                             ("pcg_sgs", "pcg", {}), ("cg", "cg", {})):
        plan = pg.Plan(pg.cart_grid(n), pg.options(method, lmax=lmax, max_iter=100000, **kw), device=dev)
        phi = torch.zeros_like(rho)
        sec, res = _time_solves(plan, rho, phi, tol, args.steps, args.warmup)
        got = phi.cpu().numpy()
        rows.append({"solver": name, "iterations": res.iterations, "time_to_1e-10_ms": sec * 1e3,
                     "gzups_per_iteration": (n - 1) ** 3 * res.iterations / (res.t_iter_ms * 1e-3) / 1e9,
                     "err_vs_oracle_rel_l2": float(np.linalg.norm(got[s, s, s] - exact[s, s, s]) /
                                                   np.linalg.norm(exact[s, s, s])),
                     "err_vs_analytic_rel_l2": float(np.linalg.norm(got[s, s, s] - ana) / np.linalg.norm(ana))})
        del plan
    cg = rows[-1]
    # preconditioned against plain CG where the grid is large enough for the
    # per-iteration cost to matter: 255^3 unknowns, C2's clump density
    big = W.config_c2(n=256, device=dev)
    study = []
    for method in ("cg", "pcg"):
        plan = pg.Plan(pg.cart_grid(256), pg.options(method, lmax=8, max_iter=20000, check_every=10), device=dev)
        phi = torch.zeros_like(big.rho)
        sec, res = _time_solves(plan, big.rho.contiguous(), phi, 1e-8, 1, 1)
        study.append({"solver": method, "iterations": res.iterations, "converged": res.converged,
                      "time_to_1e-8_ms": sec * 1e3, "ms_per_iteration": res.t_iter_ms / max(1, res.iterations)})
        del plan, phi
    out = {
        "metric": "Gcell-updates/s", "value": (n - 1) ** 3 * cg["iterations"] / (cg["time_to_1e-10_ms"] * 1e-3) / 1e9,
        "unit": "Gcell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": cg["time_to_1e-10_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "c1_uniform_sphere_32^3_lmax4_cg_and_sor_tol1e-10", "unknowns": (n - 1) ** 3},
        "rows": rows, "cg_vs_pcg_255": study,
    }
    print(json.dumps(out), flush=True)


def progress(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_description() -> dict:
    """Host cores and CPU model of the machine the oracle runs on."""
    model = None
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.lower().startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        model = None
    if model is None:
        try:
            for line in open("/proc/cpuinfo"):
                if line.lower().startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    return {"os_cpu_count": os.cpu_count(), "usable_cpus": affinity, "cpu_model": model}


def _timed_solves(plan, rho, phi, tol, steps, warmup):
    """warmup untimed cold-start solves, then `steps` timed ones bracketed by
    device synchronisation; per-solve wall latencies (each solve ends with the
    library's own convergence read-back, so they add up to the total)."""
    import torch
    res = None
    for _ in range(warmup):
        phi.zero_()
        res = plan.solve(rho, phi, tol=tol)
    torch.cuda.synchronize()
    lats, its, tmp, tit = [], [], [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        t1 = time.perf_counter()
        phi.zero_()
        res = plan.solve(rho, phi, tol=tol)
        torch.cuda.synchronize()
        lats.append(time.perf_counter() - t1)
        if not res.converged:
            raise RuntimeError(f"solve did not converge: {res}")
        its.append(res.iterations)
        tmp.append(res.t_multipole_ms)
        tit.append(res.t_iter_ms)
    sec = (time.perf_counter() - t0) / steps
    return sec, res, {"lat_ms": [x * 1e3 for x in lats], "iterations": its, "t_multipole_ms": tmp,
                      "t_iter_ms": tit}


def _pass_ms(plan, passes_per_sweep: int, sweeps: int = 20) -> float:
    """Average duration of one fine-level colour pass, HIP events on the
    plan's stream around `sweeps` resident sweeps."""
    import torch

    import paper_2605_03563_amd as pg
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    pg.sweep_resident(plan, 2)
    ev0.record(plan.stream)
    pg.sweep_resident(plan, sweeps)
    ev1.record(plan.stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / (passes_per_sweep * sweeps)


def _rel_l2(a, b) -> float:
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _oracle_errors(label, n, g, order, rho_dev, runs):
    """Errors of GPU solves against the oracle's exact discrete solution of
    the same input (its own multipole ghosts, FP64 on the host).  runs:
    {name: phi tensor}; returns {name: rel L2 error over the unknowns}."""
    from oracle import direct as OD
    from oracle import multipole as OM
    progress(f"{label}: oracle multipole boundary and exact solve at {n - 1}^3")
    t0 = time.perf_counter()
    rho = rho_dev.cpu().numpy()
    ghost, _ = OM.cart_boundary(rho, n, g, 8)
    exact = OD.solve_cart(ghost, rho, n, 1.0 / n, order, g)
    s = slice(g, g + n - 1)
    ref = exact[s, s, s]
    out = {name: _rel_l2(phi.cpu().numpy()[s, s, s], ref) for name, phi in runs.items()}
    out["oracle_seconds"] = time.perf_counter() - t0
    return out


def _accuracy_leg(label, n, g, order, rho, oracle, tol):
    """FP64 and mixed multigrid on one input, stopped at tol and driven to
    1e-12, each compared with the oracle."""
    import torch

    import paper_2605_03563_amd as pg
    grid = pg.cart_grid(n, ghost=g)
    runs, info = {}, {}
    for method in ("mg", "mg_ir32"):
        plan = pg.Plan(grid, pg.options(method, order=order, lmax=8), device="cuda:0")
        for t in (tol, 1e-12):
            phi = torch.zeros_like(rho)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = plan.solve(rho, phi, tol=t)
            torch.cuda.synchronize()
            key = f"{method}_tol{t:g}"
            runs[key] = phi
            info[key] = {"iterations": r.iterations, "rel_residual": r.rel_residual, "converged": r.converged,
                         "ms": (time.perf_counter() - t0) * 1e3}
        del plan
    if oracle:
        errs = _oracle_errors(label, n, g, order, rho, runs)
        for k in runs:
            info[k]["err_vs_oracle_rel_l2"] = errs[k]
        info["oracle_seconds"] = errs["oracle_seconds"]
    return info


def _serving_leg(n_requests: int):
    """A short request stream (sizes 32^3..256^3, warm starts): saturation
    throughput of the full server and of the FIFO FP64 cold-start baseline,
    then both at 0.7x the baseline's own saturation, where it can keep up,
    with p50 / p99 latency from arrival to completion."""
    import torch

    import paper_2605_03563_amd as pg
    import workloads as W
    dev = "cuda:0"
    reqs = W.serving_stream(n_requests=n_requests, rate=1.0, seed=5)
    rhos = [r.density(dev) for r in reqs]
    torch.cuda.synchronize()
    budget = 64 << 30

    def run(cfg, rate):
        phis = [torch.zeros_like(x) for x in rhos]
        srv = pg.Server(budget, **cfg)
        seen = {}
        for r, x in zip(reqs, rhos):
            if r.n not in seen:
                seen[r.n] = (x, torch.zeros_like(x))
        for i, (n, (x, y)) in enumerate(seen.items()):
            st = srv.wait(srv.submit(-1 - i, n, x, y))
            if st != 0:
                raise RuntimeError(f"warm-up request failed with status {st}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tickets = []
        for r, x, y in zip(reqs, rhos, phis):
            if rate is not None:
                target = t0 + r.arrival / rate
                while True:
                    dt = target - time.perf_counter()
                    if dt <= 0:
                        break
                    time.sleep(min(dt, 0.0005) if dt > 0.0002 else 0)
            tickets.append(srv.submit(r.stream_id, r.n, x, y))
        stats = []
        for t in tickets:
            st = srv.wait(t, 600000.0)
            if st != 0:
                raise RuntimeError(f"request failed with status {st}")
            stats.append(srv.poll(t))
        wall = time.perf_counter() - t0
        srv.close()
        lat = [l for _, l in stats]
        return {"solves_per_s": len(reqs) / wall, "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99),
                "mean_steps": statistics.mean(s.iterations for s, _ in stats)}

    full = dict(max_slots=8, mixed=True, warm_start=True, use_graphs=True)
    fifo = dict(max_slots=1, mixed=False, warm_start=False, use_graphs=False)
    sat_full = run(full, None)
    sat_fifo = run(fifo, None)
    rate = 0.7 * sat_fifo["solves_per_s"]
    at_full = run(full, rate)
    at_fifo = run(fifo, rate)
    return {"requests": n_requests, "sizes": "32^3-256^3 (weights 0.4/0.3/0.2/0.1)",
            "offered_rate_per_s": rate, "offered_load": "0.7x the FIFO FP64 baseline's saturation",
            "full": at_full, "fifo_fp64_cold": at_fifo,
            "speedup_p50_vs_fifo_fp64": at_fifo["p50_ms"] / at_full["p50_ms"],
            "speedup_p99_vs_fifo_fp64": at_fifo["p99_ms"] / at_full["p99_ms"],
            "saturation_solves_per_s": {"full": sat_full["solves_per_s"], "fifo_fp64_cold": sat_fifo["solves_per_s"]}}


def hbm_ceiling(gib: float = 2.0, reps: int = 10) -> dict:
    """Plain streams on the same device, on arrays of `gib` GiB each (beyond
    the 256 MB Infinity Cache): a read-only sum, a copy and a triad
    c = a + s b (two reads, one write: a colour pass's stream mix), timed
    with events; torch's own kernels, for context beside the roofline."""
    import torch
    n = int(gib * (1 << 30)) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.ones_like(a)
    c = torch.empty_like(a)
    out = {"array_GiB": gib}
    for name, fn, nbytes in (("read_GBps", lambda: a.sum(), 8 * n),
                             ("copy_GBps", lambda: c.copy_(a), 16 * n),
                             ("triad_GBps", lambda: torch.add(a, b, alpha=0.5, out=c), 24 * n)):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b, c
    return out


def bench_c3(args):
    """Default line: 512^3 intervals (511^3 unknowns), 19-point 6th-order star,
    64 Gaussian clumps + 5% lognormal |k|^-2 floor, lmax 8: all-FP64 four-colour
    multigrid V(2,2) to 1e-8 from a cold start, beside the FP32 multigrid in
    FP64 iterative refinement on the same input."""
    import torch

    import paper_2605_03563_amd as pg
    import workloads as W

    dev = "cuda:0"
    n = args.n or 512
    unknowns = (n - 1) ** 3
    progress(f"c3 density at {n}^3 intervals")
    wl = W.config_c3(n=n, device=dev)
    rho = wl.rho.contiguous()
    del wl
    grid = pg.cart_grid(n, ghost=3)

    progress("FP64 19-point multigrid")
    p64 = pg.Plan(grid, pg.options("mg", order=6, lmax=8), device=dev)
    phi = torch.zeros_like(rho)
    sec, r64, rec = _timed_solves(p64, rho, phi, args.tol, args.steps, args.warmup)
    # the FP64 19-point multigrid stops on the residual its cycles form after
    # the pre-smoothing: the last cycle begun ends there and counts as the
    # half (nu1 of nu1 + nu2 sweeps) it runs
    cycles_begun = statistics.mean(rec["iterations"])
    cycles = cycles_begun - 0.5
    value = unknowns * cycles / sec / 1e9
    pass_ms = _pass_ms(p64, 4)
    bytes_per_pass = 10.0 * unknowns   # FP64: three other colours and f_c read, colour c written
    achieved = bytes_per_pass / (pass_ms * 1e-3) / 1e9
    traffic = traffic_from_profiles("pass19v_f64_c3_511")
    del p64

    mixed = None
    if not args.no_mixed:
        progress("FP32 19-point multigrid in FP64 refinement")
        p32 = pg.Plan(grid, pg.options("mg_ir32", order=6, lmax=8), device=dev)
        sec32, r32, rec32 = _timed_solves(p32, rho, phi, args.tol, args.steps, args.warmup)
        pass32_ms = _pass_ms(p32, 4)
        mixed = {"time_to_1e-8_ms": sec32 * 1e3, "refinement_steps": statistics.mean(rec32["iterations"]),
                 "speedup_vs_fp64_mg": sec / sec32, "rel_residual": r32.rel_residual,
                 "p50_ms": _pct(rec32["lat_ms"], 50), "p99_ms": _pct(rec32["lat_ms"], 99),
                 "fine_pass_fp32_ms": pass32_ms,
                 "fine_pass_fp32_GBps": 5.0 * unknowns / (pass32_ms * 1e-3) / 1e9}
        del p32
    del phi, rho

    progress("7-point FP64 colour pass at 511^3")
    w7 = W.config_c2(n=512, device=dev)
    rho7 = w7.rho.contiguous()
    del w7
    p7 = pg.Plan(pg.cart_grid(512), pg.options("mg", lmax=8), device=dev)
    phi7 = torch.zeros_like(rho7)
    r7 = p7.solve(rho7, phi7, tol=args.tol)
    pass7_ms = _pass_ms(p7, 2)
    pass7 = {"pass_ms": pass7_ms, "algorithmic_bytes_per_launch": 12.0 * unknowns,
             "GBps": 12.0 * unknowns / (pass7_ms * 1e-3) / 1e9,
             "frac": 12.0 * unknowns / (pass7_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
             "gcell_updates_per_s": unknowns / (2 * pass7_ms * 1e-3) / 1e9,
             "traffic": traffic_from_profiles("rb_pass7v_f64_c2_511"),
             "kernel": "k_pass7v<double, 2> (fine-level red-black GS colour pass)",
             "solve": {"v_cycles": r7.iterations, "ms": r7.t_multipole_ms + r7.t_iter_ms}}
    del p7, phi7, rho7

    ceiling = hbm_ceiling()

    oracle = not args.no_oracle_errors
    progress("255^3 clump workload (7-point), FP64 and mixed, against the oracle")
    w2 = W.config_c2(n=256, device=dev)
    acc_c2 = _accuracy_leg("c2", 256, 1, 2, w2.rho.contiguous(), oracle, args.tol)
    del w2
    progress("19-point workload at 255^3, FP64 and mixed, against the oracle")
    w3 = W.config_c3(n=256, device=dev)
    acc_c3 = _accuracy_leg("c3@256", 256, 3, 6, w3.rho.contiguous(), oracle, args.tol)
    del w3

    serving = None
    if args.serve_requests > 0:
        progress(f"serving leg, {args.serve_requests} requests")
        serving = _serving_leg(args.serve_requests)

    cpu = None
    if not args.no_cpu_baseline:
        progress("CPU oracle baseline")
        cpu = cpu_baseline_c3(args.cpu_budget_s)

    out = {
        "metric": "Gcell-updates/s", "value": value, "unit": "Gcell-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"c3_clumps64_floor_{n}^3_star19_fp64_mg_v22_4colour_gs_lmax8_tol{args.tol:g}",
                   "unknowns": unknowns, "solver": "MG V(2,2) four-colour GS on the 19-point star, FW "
                   "restriction, trilinear prolongation, 7^3 exact coarsest", "parallelism": "single-gpu"},
        "time_to_1e-8_ms": sec * 1e3,
        "time_to_1e-8_p50_ms": _pct(rec["lat_ms"], 50), "time_to_1e-8_p99_ms": _pct(rec["lat_ms"], 99),
        "time_to_1e-8_median_device_ms": statistics.median(a + b for a, b in zip(rec["t_multipole_ms"],
                                                                                 rec["t_iter_ms"])),
        "v_cycles": cycles, "v_cycles_begun": cycles_begun, "rate": r64.rate, "rel_residual": r64.rel_residual,
        "t_multipole_ms": statistics.mean(rec["t_multipole_ms"]), "t_iter_ms": statistics.mean(rec["t_iter_ms"]),
        "s_s_gzups": unknowns / (statistics.mean(rec["t_iter_ms"]) / cycles * 1e-3) / 1e9,
        "s_t_gzups": unknowns / sec / 1e9,
        "fine_pass_ms": pass_ms,
        "fine_pass_gcell_updates_per_s": unknowns / (4 * pass_ms * 1e-3) / 1e9,
        "copy_GBps": ceiling["copy_GBps"],
        "hbm_ceiling": ceiling,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": "k_pass19v<double, 2> (fine-level four-colour GS pass)",
                     "algorithmic_bytes_per_launch": bytes_per_pass},
        "mixed_fp32_mg_in_fp64_ir": mixed,
        "rb_pass7_f64_511": pass7,
        "accuracy_vs_oracle_255": {"c2_clumps16_7pt": acc_c2, "c3_recipe_19pt": acc_c3},
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def c4(args):
    """Log-spherical 256 x 128 x 256 grid (r in [1e-3, 1]), truncated SIS with a
    10% m = 2 perturbation, lmax 8 outer + inner expansions and the excised
    core as a central point mass; FP64 BiCGSTAB from a cold start, right-
    preconditioned by one FP32 multigrid V(2,2) cycle, beside the red-black
    Gauss-Seidel preconditioner, spherical SOR, and the same core on the
    padded radial grid."""
    import torch

    import paper_2605_03563_amd as pg
    import workloads as W

    dev = "cuda:0"
    wl = W.config_c4(device=dev)
    rho = wl.rho.contiguous()
    g = wl.grid
    grid = pg.sph_grid(g.nr, g.nth, g.nph)
    unknowns = g.unknowns
    runs = {}
    for m in ("bicgstab_mg32", "bicgstab"):
        plan = pg.Plan(grid, pg.options(m, lmax=8, point_mass=4 * math.pi * g.r_min, max_iter=20000,
                                        check_every=10 if m == "bicgstab" else 1), device=dev)
        phi = torch.zeros_like(rho)
        steps = max(1, args.steps // 2) if m == "bicgstab" else args.steps
        sec, res = _time_solves(plan, rho, phi, args.tol, steps, 1)
        runs[m] = (sec, res, steps)
        del plan, phi
    # SOR with the local Chebyshev relaxation sequence (Eq. local_rjac), one solve
    plan = pg.Plan(grid, pg.options("sor", lmax=8, point_mass=4 * math.pi * g.r_min, max_iter=40000,
                                    check_every=50, omega_mode=pg.OMEGA_CHEBYSHEV), device=dev)
    phi = torch.zeros_like(rho)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rsor = plan.solve(rho, phi, tol=args.tol)
    torch.cuda.synchronize()
    ssor = time.perf_counter() - t0
    del plan, phi
    # the same core with the padding of Section 3.3: 20 inner cells along the
    # quartic down to r_min / 2 and 20 outer log cells, density zero in the
    # pads (the core's density copied in); BiCGSTAB with the Gauss-Seidel
    # preconditioner; then with the FP32 multigrid one, whose levels need a
    # radial count that halves five times: 14 outer cells (288 unknowns)
    def padded(method, ext_in, ext_out, check_every):
        nr_pad = g.nr + (ext_in - 1) + (ext_out - 1)
        gpad = pg.sph_grid(nr_pad, g.nth, g.nph, g.r_min, g.r_max, ext_in=ext_in, ext_out=ext_out,
                           r_pad=g.r_min / 2)
        rho_pad = torch.zeros((g.nph, g.nth, nr_pad + 2), dtype=torch.float64, device=dev)
        rho_pad[:, :, ext_in:ext_in + g.nr] = rho[:, :, 1:g.nr + 1]
        plan = pg.Plan(gpad, pg.options(method, lmax=8, point_mass=4 * math.pi * g.r_min, max_iter=20000,
                                        check_every=check_every), device=dev)
        phi = torch.zeros_like(rho_pad)
        sp, rp = _time_solves(plan, rho_pad, phi, args.tol, 1, 1)
        return {"radial_unknowns": nr_pad, "ext_in": ext_in, "ext_out": ext_out, "r_pad": g.r_min / 2,
                "time_to_1e-8_ms": sp * 1e3, "iterations": rp.iterations, "converged": rp.converged,
                "ms_per_iteration": rp.t_iter_ms / max(1, rp.iterations)}
    pad_gs = padded("bicgstab", 20, 20, 10)
    pad_mg = padded("bicgstab_mg32", 20, 14, 1)
    sec, res, steps = runs["bicgstab_mg32"]
    sgs, rgs, _ = runs["bicgstab"]
    gs_it_ms = rgs.t_iter_ms / max(1, rgs.iterations)
    bytes_per_it = 200.0 * unknowns   # Gauss-Seidel-preconditioned iteration: 7 streaming kernels
    out = {
        "metric": "Gcell-updates/s", "value": unknowns * res.iterations / sec / 1e9, "unit": "Gcell-updates/s",
        "n_gpus": 1, "steps": steps, "warmup": 1, "ms_per_step": sec * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": "c4_sis_m2_256x128x256_logsph_bicgstab_fp32mg_lmax8", "unknowns": unknowns},
        "time_to_1e-8_ms": sec * 1e3, "iterations": res.iterations, "rel_residual": res.rel_residual,
        "t_multipole_ms": res.t_multipole_ms, "ms_per_iteration": res.t_iter_ms / max(1, res.iterations),
        "gs_preconditioned": {"time_to_1e-8_ms": sgs * 1e3, "iterations": rgs.iterations,
                              "ms_per_iteration": gs_it_ms,
                              "iteration_GBps_algorithmic": bytes_per_it / (gs_it_ms * 1e-3) / 1e9},
        "speedup_mg_vs_gs": sgs / sec,
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline_c4(rho.cpu().numpy(), g, args.cpu_budget_s),
        "sor_local_chebyshev": {"time_ms": ssor * 1e3, "converged": rsor.converged, "sweeps": rsor.iterations,
                                "rel_residual": rsor.rel_residual,
                                "ms_per_sweep": rsor.t_iter_ms / max(1, rsor.iterations)},
        "padded_grid_gs_bicgstab": pad_gs,
        "padded_grid_fp32mg_bicgstab": pad_mg,
    }
    print(json.dumps(out), flush=True)


def spai(args):
    """The paper's own multigrid (Table 2 shape): 512^3 intervals (511^3
    unknowns), seven coarse levels (coarsest 4 intervals), SPAI Richardson
    smoothing with the Table 1 coefficients, Galerkin coarse operators,
    compact stencils of order 2, 4 and 6, V(nu, nu) for nu = 1, 2, 3, FP64 and
    FP32 coarse-level storage; density of 64 clumps and the turbulent floor
    (the 512^3 workload), multipole boundary lmax 8, cold start, tol 1e-8.
    Reports the time per V-cycle s and the mean rate rho of Eq. rho beside
    the paper's Table 2 values (other hardware: context only)."""
    import torch

    import paper_2605_03563_amd as pg
    import workloads as W

    dev = "cuda:0"
    n = 512
    wl = W.config_c3(n=n, device=dev, g=1)
    rho = wl.rho.contiguous()
    del wl
    # order 6 reads the density's second ghost layer: the same recipe on a
    # two-ghost grid
    wl = W.config_c3(n=n, device=dev, g=2)
    rho6 = wl.rho.contiguous()
    del wl
    unknowns = (n - 1) ** 3
    grid = pg.cart_grid(n, ghost=1)
    grid6 = pg.cart_grid(n, ghost=2)
    paper = {(2, 1): (3.48e-2, 0.102), (2, 2): (5.29e-2, 0.028), (2, 3): (7.27e-2, 0.013),
             (4, 1): (3.49e-2, 0.065), (4, 2): (5.33e-2, 0.017), (4, 3): (7.37e-2, 0.011),
             (6, 1): (3.53e-2, 0.068), (6, 2): (5.46e-2, 0.018), (6, 3): (7.47e-2, 0.012)}
    rows = []
    best = None
    for method in ("mg_spai", "mg_spai32"):
        for order in (2, 4, 6):
            for nu in (1, 2, 3):
                g_o, rho_o = (grid6, rho6) if order == 6 else (grid, rho)
                plan = pg.Plan(g_o, pg.options(method, order=order, lmax=8, nu1=nu, nu2=nu, coarsest=4), device=dev)
                phi = torch.zeros_like(rho_o)
                sec, res = _time_solves(plan, rho_o, phi, args.tol, max(1, args.steps // 2), 1)
                s_cycle = res.t_iter_ms / max(1, res.iterations) * 1e-3
                row = {"method": method, "order": order, "nu": nu, "cycles": res.iterations,
                       "time_to_1e-8_ms": sec * 1e3, "s_per_cycle": s_cycle, "rho": res.rate,
                       "s_times_rho": s_cycle * res.rate, "t_multipole_ms": res.t_multipole_ms,
                       "paper_s": paper[(order, nu)][0], "paper_rho": paper[(order, nu)][1]}
                rows.append(row)
                print(json.dumps({"spai_row": row}), flush=True)
                if method == "mg_spai32" and order == 2 and nu == 3:
                    best = (plan, row, sec)
                else:
                    del plan
    # coarsest solve: dense inverse against CG to relative accuracy rho (Section 2.1.3)
    coarse_rows = []
    for coarsest, ctol in ((4, 0.0), (4, 0.013), (8, 0.0), (8, 0.013)):
        p2 = pg.Plan(grid, pg.options("mg_spai", order=2, lmax=8, nu1=3, nu2=3, coarsest=coarsest,
                                      coarse_tol=ctol), device=dev)
        phi = torch.zeros_like(rho)
        sec2, res2 = _time_solves(p2, rho, phi, args.tol, max(1, args.steps // 2), 1)
        coarse_rows.append({"coarsest": coarsest, "coarse_solve": "cg" if ctol > 0 else "dense",
                            "coarse_tol": ctol, "cycles": res2.iterations, "rho": res2.rate,
                            "s_per_cycle": res2.t_iter_ms / max(1, res2.iterations) * 1e-3,
                            "time_to_1e-8_ms": sec2 * 1e3})
        print(json.dumps({"spai_coarse_row": coarse_rows[-1]}), flush=True)
        del p2
    plan, row, sec = best
    # dominant kernels: the fine-level residual and smoother stencils (one SPAI
    # step = both), timed resident on the plan's stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    pg.sweep_resident(plan, 1)
    ev0.record(plan.stream)
    pg.sweep_resident(plan, 10)
    ev1.record(plan.stream)
    torch.cuda.synchronize()
    step_ms = ev0.elapsed_time(ev1) / 20     # sweep_resident(k) = 2k fused steps
    bytes_per_step = 24.0 * unknowns   # fused SPAI step: read u, f; write the new u (FP64)
    achieved = bytes_per_step / (step_ms * 1e-3) / 1e9
    out = {
        "metric": "Gcell-updates/s", "value": unknowns * row["cycles"] / sec / 1e9, "unit": "Gcell-updates/s",
        "n_gpus": 1, "steps": max(1, args.steps // 2), "warmup": 1, "ms_per_step": sec * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32storage",
        "data": "synthetic",
        "config": {"workload": "spai_mg_512^3_order2_V33_fp32coarse_lmax8", "unknowns": unknowns},
        "time_to_1e-8_ms": sec * 1e3, "cycles": row["cycles"], "rows": rows, "coarse_rows": coarse_rows,
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline_spai(args.cpu_budget_s),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic_from_profiles("spai_step_f64_511"),
                     "kernel": "k_nspai<double, 16> (fused fine-level SPAI step)",
                     "algorithmic_bytes_per_launch": bytes_per_step, "step_ms": step_ms},
    }
    print(json.dumps(out), flush=True)


def serving(args):
    """Serving stream: Poisson arrivals over 64 stream ids, sizes 32^3..256^3
    (weights 0.4/0.3/0.2/0.1), 1-32 clumps per stream, each request a small
    perturbation of its stream's previous one; mixed-precision multigrid to
    1e-8 with warm starts, graph-launched steps and continuous batching."""
    import torch

    import paper_2605_03563_amd as pg
    import workloads as W

    dev = "cuda:0"
    reqs = W.serving_stream(n_requests=args.requests, rate=1.0, seed=5)
    rhos = [r.density(dev) for r in reqs]
    torch.cuda.synchronize()
    budget = int(args.budget_gb * (1 << 30))

    def run(cfg, rate):
        phis = [torch.zeros_like(x) for x in rhos]
        srv = pg.Server(budget, **cfg)
        for n in sorted(set(r.n for r in reqs)):
            srv.reserve(n, cfg["max_slots"])
        # warm the plan pool and graphs with one request per size on spare stream ids
        seen = {}
        for r, x in zip(reqs, rhos):
            if r.n not in seen:
                seen[r.n] = (x, torch.zeros_like(x))
        for i, (n, (x, y)) in enumerate(seen.items()):
            srv.wait(srv.submit(-1 - i, n, x, y))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tickets = []
        for r, x, y in zip(reqs, rhos, phis):
            if rate is not None:
                target = t0 + r.arrival / rate
                while True:
                    dt = target - time.perf_counter()
                    if dt <= 0:
                        break
                    time.sleep(min(dt, 0.0005) if dt > 0.0002 else 0)
            tickets.append(srv.submit(r.stream_id, r.n, x, y))
        stats = []
        for t in tickets:
            st = srv.wait(t, 600000.0)
            if st != 0:
                raise RuntimeError(f"request failed with status {st}")
            stats.append(srv.poll(t))
        wall = time.perf_counter() - t0
        srv.close()
        lat = [l for _, l in stats]
        its = [s.iterations for s, _ in stats]
        return {"solves_per_s": len(reqs) / wall, "wall_s": wall, "p50_ms": _pct(lat, 50),
                "p99_ms": _pct(lat, 99), "mean_steps": statistics.mean(its),
                "converged": sum(1 for s, _ in stats if s.status == 0)}

    full = dict(max_slots=args.slots, mixed=True, warm_start=True, use_graphs=True)
    sat = run(full, None)
    rate = args.load * sat["solves_per_s"]
    configs = {
        "fifo_fp64_cold_nographs": dict(max_slots=1, mixed=False, warm_start=False, use_graphs=False),
        "+warm_start": dict(max_slots=1, mixed=False, warm_start=True, use_graphs=False),
        "+mixed_precision": dict(max_slots=1, mixed=True, warm_start=True, use_graphs=False),
        "+graphs": dict(max_slots=1, mixed=True, warm_start=True, use_graphs=True),
        "+batching(full)": full,
    }
    res = {k: run(v, rate) for k, v in configs.items()}
    base, best = res["fifo_fp64_cold_nographs"], res["+batching(full)"]
    out = {
        "metric": "solves/s at offered load; p50/p99 latency", "value": best["solves_per_s"],
        "unit": "solves/s", "n_gpus": 1, "steps": len(reqs), "warmup": len(set(r.n for r in reqs)),
        "ms_per_step": best["wall_s"] * 1e3 / len(reqs), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"serving_{len(reqs)}req_sizes32-256_poisson_arrivals_{args.load:g}x_saturation",
                   "offered_rate_per_s": rate, "budget_gb": args.budget_gb},
        "p50_ms": best["p50_ms"], "p99_ms": best["p99_ms"],
        "saturation": sat,
        "speedup_p99_vs_fifo_fp64": base["p99_ms"] / best["p99_ms"],
        "speedup_p50_vs_fifo_fp64": base["p50_ms"] / best["p50_ms"],
        "ablations": res,
    }
    print(json.dumps(out), flush=True)


def kernels_only(args):
    """Dispatch the dominant kernel and a copy kernel of known size so that
    rocprofv3 counters (FETCH_SIZE, WRITE_SIZE) can be read per dispatch:
    c3: the FP64 four-colour pass at 511^3 (19-point star); c2: the FP64
    red-black pass (7-point, --n intervals, default 512); spai: the fused SPAI
    step at 511^3."""
    import torch

    import paper_2605_03563_amd as pg
    import workloads as W

    dev = "cuda:0"
    if args.workload == "spai":
        # the fused SPAI step at 511^3 (one V(1,1) cycle's solve, then resident steps)
        wl = W.config_c3(n=512, device=dev, g=1)
        rho = wl.rho.contiguous()
        plan = pg.Plan(pg.cart_grid(512), pg.options("mg_spai", order=2, lmax=8, nu1=1, nu2=1, coarsest=4,
                                                      max_iter=1), device=dev)
        what = "fused SPAI steps"
    elif args.workload == "c3":
        n = args.n or 512
        wl = W.config_c3(n=n, device=dev)
        rho = wl.rho.contiguous()
        plan = pg.Plan(pg.cart_grid(n, ghost=3), pg.options("mg", order=6, lmax=8, max_iter=1), device=dev)
        what = "four-colour sweeps"
    else:
        n = args.n or 512
        wl = W.config_c2(n=n, device=dev)
        rho = wl.rho.contiguous()
        plan = pg.Plan(pg.cart_grid(n), pg.options("mg", lmax=8, max_iter=1), device=dev)
        what = "red-black sweeps"
    del wl
    phi = torch.zeros_like(rho)
    plan.solve(rho, phi, tol=args.tol)
    pg.sweep_resident(plan, args.sweeps)
    a = torch.ones(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"kernels-only ({args.workload}): {args.sweeps} {what}, copy of {a.numel() * 8} bytes", flush=True)


def traffic_from_profiles(kernel_tag: str):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, when it was taken on the current kernel."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    try:
        return float(vals["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(rho_host, n, budget_s, with_multipole):
    from threadpoolctl import threadpool_limits

    from oracle import multipole as OM
    from oracle import smoothers as OS

    unknowns = (n - 1) ** 3
    with threadpool_limits(limits=1):
        t_mp = None
        if with_multipole:
            t0 = time.perf_counter()
            ghost, _ = OM.cart_boundary(rho_host, n, 1, 8)
            t_mp = time.perf_counter() - t0
        else:
            ghost = rho_host * 0.0
        u = ghost.copy()
        cache = {}
        cycles = 0
        t0 = time.perf_counter()
        while True:
            OS.vcycle(u, rho_host, n, 1.0 / n, 2, 1, _cache=cache)
            cycles += 1
            el = time.perf_counter() - t0
            if el >= budget_s:
                break
    sample = (f"{cycles} V(2,2) cycle(s) of the oracle's NumPy reference V-cycle on the same "
              f"{n - 1}^3-unknown input, single thread, {el:.1f} s")
    if t_mp is not None:
        sample += f"; oracle multipole boundary (lmax 8) took {t_mp:.1f} s (not in value)"
    return {"value": unknowns * cycles / el / 1e9, "unit": "Gcell-updates/s", "cores": 1,
            "kind": "oracle", "sample": sample, "host": host_description()}


def _cpu_repeat(fn, budget_s):
    """Run fn() single-threaded until budget_s has elapsed (at least once);
    returns (calls, seconds)."""
    from threadpoolctl import threadpool_limits
    calls = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while True:
            fn()
            calls += 1
            el = time.perf_counter() - t0
            if el >= budget_s:
                break
    return calls, el


def cpu_baseline_c3(budget_s):
    """Oracle 19-point V(2,2) cycles on the same workload recipe at 128^3
    (64 clumps + turbulent floor), single thread."""
    from oracle import smoothers as OS
    import workloads as W
    n, g = 128, 3
    wl = W.config_c3(n=n, g=g)
    rho = wl.rho.numpy()
    u = np.zeros_like(rho)
    cache = {}
    calls, el = _cpu_repeat(lambda: OS.vcycle(u, rho, n, 1.0 / n, 6, g, _cache=cache), budget_s)
    return {"value": (n - 1) ** 3 * calls / el / 1e9, "unit": "Gcell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{calls} oracle 19-point V(2,2) cycle(s) (FP64 NumPy) on the same recipe at 128^3 "
                      f"(127^3 unknowns), single thread, {el:.1f} s", "host": host_description()}


def cpu_baseline_c4(rho_host, g, budget_s):
    """Oracle r^2-scaled spherical operator (residual) applications on the
    full C4 input, single thread."""
    from oracle import multipole as OM
    from oracle import operators as OO
    r, th, ph, ds = OM.sph_axes(g.nr, g.nth, g.nph)
    u = np.zeros_like(rho_host)
    calls, el = _cpu_repeat(lambda: OO.sph_residual(u, rho_host, r, ds, th), budget_s)
    return {"value": g.unknowns * calls / el / 1e9, "unit": "Gcell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{calls} oracle residual evaluation(s) of the r^2-scaled spherical operator on the full "
                      f"{g.nr}x{g.nth}x{g.nph} input, single thread, {el:.1f} s (the oracle solves C4 directly; "
                      f"this is its per-sweep building block)", "host": host_description()}


def cpu_baseline_spai(budget_s):
    """Oracle SPAI V(3,3) cycles (order 2, Galerkin levels) on the same
    recipe at 128^3, single thread."""
    from oracle import spai as SP
    import workloads as W
    n = 128
    wl = W.config_c3(n=n, g=1)
    rho = wl.rho.numpy()
    ops = SP.level_operators(2, n, 4)
    f = SP.rhs_compact(rho, n, 2)
    u = np.zeros_like(rho)
    cache = {}
    calls, el = _cpu_repeat(lambda: SP.vcycle(u, f, n, ops, SP.COEFFS[2], 3, 3, _cache=cache), budget_s)
    return {"value": (n - 1) ** 3 * calls / el / 1e9, "unit": "Gcell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{calls} oracle SPAI V(3,3) cycle(s) (order 2, Galerkin coarse levels to 4 intervals) on "
                      f"the same recipe at 128^3, single thread, {el:.1f} s", "host": host_description()}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the solver runs on one MI355X; --gpus above 1 is not supported "
              "(sharding over several GPUs is designed but not implemented)", file=sys.stderr)
        sys.exit(2)

    if args.kernels_only:
        kernels_only(args)
        return
    if args.workload != "c2":
        {"serving": serving, "c1": bench_c1, "c3": bench_c3, "c4": c4, "spai": spai}[args.workload](args)
        return
    bench_c2(args)


def bench_c2(args):
    """256^3 intervals (255^3 unknowns), 16 Gaussian clumps, 7-point operator,
    lmax 8: FP64 multigrid V(2,2) with red-black Gauss-Seidel to 1e-8."""
    import torch

    import paper_2605_03563_amd as pg
    import workloads as W

    dev = "cuda:0"
    n = args.n or 256
    unknowns = (n - 1) ** 3
    wl = W.config_c2(n=n, device=dev)
    rho = wl.rho.contiguous()
    grid = pg.cart_grid(n)
    plan = pg.Plan(grid, pg.options("mg", lmax=8), device=dev)
    phi = torch.zeros_like(rho)

    def run(p, steps):
        its, t_mp, t_it, rels = [], [], [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            phi.zero_()
            r = p.solve(rho, phi, tol=args.tol)
            if not r.converged:
                raise RuntimeError(f"solve did not converge: {r}")
            its.append(r.iterations)
            t_mp.append(r.t_multipole_ms)
            t_it.append(r.t_iter_ms)
            rels.append(r.rel_residual)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, its, t_mp, t_it, rels

    run(plan, args.warmup)
    sec, its, t_mp, t_it, rels = run(plan, args.steps)
    ms_per_step = sec * 1e3
    cycles = statistics.mean(its)
    value = unknowns * cycles / sec / 1e9

    # dominant kernel: the fine-level red-black colour pass, timed alone with
    # HIP events on the plan's stream (same arrays and launch configuration)
    sweeps = 20
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(plan.stream):
        pg.sweep_resident(plan, 2)
        ev0.record(plan.stream)
        pg.sweep_resident(plan, sweeps)
        ev1.record(plan.stream)
    torch.cuda.synchronize()
    pass_ms = ev0.elapsed_time(ev1) / (2 * sweeps)
    bytes_per_pass = 12.0 * unknowns          # FP64 GS colour pass: 24 B per unknown per full sweep
    achieved = bytes_per_pass / (pass_ms * 1e-3) / 1e9
    traffic = traffic_from_profiles("rb_pass7v_f64_c2_255")

    # plain copy bandwidth on the same device for context
    a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(10):
        b.copy_(a)
    c1.record()
    torch.cuda.synchronize()
    copy_gbps = 2 * a.numel() * 4 * 10 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del a, b

    extra = {}
    if not args.no_mixed:
        plan32 = pg.Plan(grid, pg.options("mg_ir32", lmax=8), device=dev)
        run(plan32, max(1, args.warmup))
        sec32, its32, _, _, _ = run(plan32, args.steps)
        extra["mixed_fp32_mg_in_fp64_ir"] = {
            "time_to_tol_ms": sec32 * 1e3, "refinement_steps": statistics.mean(its32),
            "speedup_vs_fp64_mg": sec / sec32}
        del plan32

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(rho.cpu().numpy(), n, args.cpu_budget_s, args.cpu_multipole)

    out = {
        "metric": "Gcell-updates/s", "value": value, "unit": "Gcell-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"c2_clumps16_{n}^3_fp64_mg_v22_rbgs_lmax8_tol{args.tol:g}",
                   "unknowns": unknowns, "solver": "MG V(2,2) red-black GS, FW restriction, "
                   "trilinear prolongation, 7^3 exact coarsest", "parallelism": "single-gpu"},
        "time_to_1e-8_ms": ms_per_step,
        "time_to_1e-8_median_device_ms": statistics.median(a + b for a, b in zip(t_mp, t_it)),
        "v_cycles": cycles,
        "t_multipole_ms": statistics.mean(t_mp),
        "t_iter_ms": statistics.mean(t_it),
        "rel_residual": max(rels),
        "s_t_gzups": unknowns / sec / 1e9,
        "smoother_pass_ms": pass_ms,
        "smoother_gcell_updates_per_s": unknowns / (2 * pass_ms * 1e-3) / 1e9,
        "copy_GBps": copy_gbps,
        # counter-measured HBM bytes of the fine pass over its event-timed duration
        "smoother_traffic_GBps": (traffic / (pass_ms * 1e-3) / 1e9) if traffic else None,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": traffic,
                     "kernel": "k_pass7v<double, 2> (fine-level red-black GS colour pass)",
                     "algorithmic_bytes_per_launch": bytes_per_pass},
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
