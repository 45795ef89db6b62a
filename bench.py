"""Benchmark of the LEM hot path on one MI355X.

Default workload: 2D periodic advection-diffusion on a 512x512 grid (velocity
(1, 0.5), nu = 1e-3, dt = 2 dx), an ensemble of 128 seeded smooth states,
32x32 cores.  Local exponentials exp(dt A_M) are computed once (float64 Pade
scaling and squaring on the GPU, excluded from the timed region and reported
as plan time) and applied every step as batched FP64 MFMA products with
fused gather and scatter.  The buffer width comes from the off-diagonal decay
bound at 1e-8 per step, so that the LEM result stays within 1e-6 (relative
l2) of the exact global exponential over the timed run; this is checked on
the GPU against the global Krylov action at 1e-13, and the global Krylov
method at 1e-8 per step is timed on the same grid as the comparator.  The
FP32 and split-bf16 applications of the same blocks, the configured 8-point
buffer and the 256x256 x 64-state workload are reported as extras.

Prints one JSON line.  A step is one full LEM step (gather, local
exponential action, core scatter) of the whole grid and ensemble.
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DOF-steps/s, LEM vs global Krylov expmv at rel err ≤1e-6; served p99 latency"
MFMA_FP64_PEAK_TFLOPS = 78.6
MFMA_FP32_PEAK_TFLOPS = 157.3
MFMA_BF16_PEAK_TFLOPS = 2500.0
HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of the FP64 apply per workload and tile shape
# (autotuner id), from rocprofv3 FETCH_SIZE / WRITE_SIZE passes scaled by a
# 256 MiB reference copy (profiles/apply_fp64_*.md); valid only for the apply
# kernel source they were taken on: the text of dense.hip from its apply
# section to the split-bf16 kernel, plus its tile-shape table.
TRAFFIC = {"c3": ("094c1b2e44e5", {0: 5924491712, 1: 5698362176, 2: 2941001920, 3: 2940792832,
                                     4: 8905402048, 5: 11436342272, 6: 5166288896,
                                     7: 2999551104})}


def _apply_source_key(text: str) -> str:
    import hashlib
    i0 = text.index("// ------------------------------------------------------------------ apply --")
    i1 = text.index("// Split-bf16 apply")
    j0 = text.index("kApplyShapes[kApplyConfigs][3] = {")
    shapes = text[j0:text.index("};", j0)]
    return hashlib.sha1((text[i0:i1] + shapes).encode()).hexdigest()[:12]


def measured_traffic(workload, tile):
    if workload not in TRAFFIC:
        return None
    src = os.path.join(ROOT, "paper_1505_02248_amd", "csrc", "dense.hip")
    key, per_tile = TRAFFIC[workload]
    with open(src) as f:
        if _apply_source_key(f.read()) != key:
            return None
    return per_tile.get(tile)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_steps(plan, x, y, k, torch):
    """Run k steps as one lem_step call; returns (wall s, event ms)."""
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(s)
    plan.step(x, y, k)
    e1.record(s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return t1 - t0, e0.elapsed_time(e1)


def host_cpu():
    """(threads BLAS uses, CPU model, logical CPUs) of this host."""
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return int(cores), model, os.cpu_count()


def cpu_baseline(p, boxes, budget_s: float, sample_blocks: int = 0, **step_kw):
    """The oracle LEM step (numpy float64) on the host cores: first the local
    exponential (excluded), then steps of the whole grid -- or of the first
    ``sample_blocks`` regions (a bounded sample; every region of these
    translation-invariant workloads costs the same) -- until ~budget_s.  The
    rate counts core points x states x steps of the regions stepped."""
    import numpy as np
    from oracle import lem as olem
    from oracle import operator as op
    from oracle import partition as P
    cores, model, ncpu = host_cpu()
    A = op.sparse(op.from_problem(p))
    bx = [P.Box(*map(int, b)) for b in boxes]
    if sample_blocks:
        bx = bx[:sample_blocks]
    core_pts = sum(b.cx * (b.cy if p.ndim == 2 else 1) for b in bx)
    ns = p.states.shape[1]
    cache = olem.LocalExpCache()
    t0 = time.perf_counter()
    olem.step(A, bx[:1], p.ndim, p.n, p.states, cache, **step_kw)  # local exponential, once
    t_plan = time.perf_counter() - t0

    def steps_for(limit_s, max_steps):
        u = p.states.copy()
        k = 0
        t0 = time.perf_counter()
        while True:
            # a sample steps its regions from the input state each time (the
            # cores outside the sample are not computed)
            u = olem.step(A, bx, p.ndim, p.n, p.states if sample_blocks else u, cache, **step_kw)
            k += 1
            el = time.perf_counter() - t0
            if el >= limit_s or k >= max_steps:
                return k, el

    steps, el = steps_for(budget_s, 200)
    what = (f"{len(bx)} of {len(boxes)} regions" if sample_blocks else f"all {len(boxes)} regions")
    how = ("the oracle's Krylov action per region" if step_kw.get("krylov_above")
           else f"one GEMM per region, local expm {t_plan:.2f} s excluded")
    out = {"value": core_pts * ns * steps / el, "unit": "DOF-steps/s", "cores": cores,
           "kind": "oracle", "cpu_model": model, "logical_cpus": ncpu,
           "sample": f"{steps} LEM steps of {what} x {ns} states (numpy float64, {how})",
           "seconds": round(el, 3)}
    # the same steps with one BLAS thread (a quarter of the time budget)
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            s1, el1 = steps_for(budget_s / 4, 50)
        out["value_1thread"] = core_pts * ns * s1 / el1
        out["sample_1thread"] = f"{s1} step{'s' if s1 > 1 else ''}, one BLAS thread"
    except ImportError:
        pass
    return out


def parse_args():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--halo-tol", type=float, default=1e-8)
    ap.add_argument("--global-steps", type=int, default=10)
    ap.add_argument("--acc-steps", type=int, default=0,
                    help="steps of the accuracy check against the global method (0: --steps)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-global", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the float32 leg of c1")
    ap.add_argument("--arms", default="fp32,bf16x3,bf16x2",
                    help="c3: reduced-precision applications timed beside FP64 (comma list, "
                         "may be empty)")
    ap.add_argument("--kron", type=int, default=1,
                    help="c3: also time the Kronecker-factored local exponentials (1/0)")
    ap.add_argument("--with-c1", type=int, default=1,
                    help="c3: also report the 256^2 x 64-state workload (1/0)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="also run one device copy of this many MiB (a reference kernel of "
                         "known traffic for scaling HBM counters)")
    ap.add_argument("--workload", default="c3", choices=["c0", "c1", "c2", "c3", "c4", "f1", "f2", "f3", "f4"],
                    help="c3 (default): 512^2 x 128 states, dense FP64 (+ FP32/bf16 arms); "
                         "c1: 256^2 x 64 states, dense FP64; c0: 1D 1024; "
                         "c2: 1024^2 lognormal nu, uneven Krylov; c4: served Poisson stream; f1: c1 with a "
                         "constant source g (exponential-Euler step with forcing); f2: "
                         "Burgers by exponential Rosenbrock-Euler LEM; f3: Schroedinger with a "
                         "harmonic potential (complex blocks in real form); f4: variable "
                         "vortex velocity and anisotropic column-wise cores (Krylov)")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--warm-requests", type=int, default=200,
                    help="c4: requests served before the measured ones")
    ap.add_argument("--krylov-m-max", type=int, default=40,
                    help="c2/c4: largest local Krylov dimension")
    ap.add_argument("--max-overhead", type=float, default=9.0,
                    help="c4: largest local/core point ratio before a request takes the "
                         "global method")
    ap.add_argument("--saturate", type=int, default=1,
                    help="c4: also time the measured requests submitted all at once (1/0)")
    ap.add_argument("--steps-per-tick", type=int, default=4, help="c4: server steps per tick")
    return ap.parse_args()


def main() -> int:
    args = parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this build "
              "(the LEM path would shard by spatial regions with one halo exchange per step, "
              "which is not implemented here)", file=sys.stderr)
        return 2
    fn = {"c1": bench_c1, "c0": bench_c0, "c2": bench_c2, "c3": bench_c3,
          "c4": bench_c4, "f1": bench_f1, "f2": bench_f2, "f3": bench_f3,
            "f4": bench_f4}[args.workload]
    out = fn(args)
    print(json.dumps(out), flush=True)
    return 0


def bench_c1(args) -> dict:
    import numpy as np
    import torch

    import lem_inputs as L
    import paper_1505_02248_amd as lem

    torch.cuda.init()
    p = L.workload_2d_ensemble()  # 256^2, 64 states
    ns = p.states.shape[1]
    opr = lem.Operator.from_problem(p)
    N = p.N
    x = torch.from_numpy(p.states.copy()).to("cuda")
    y = torch.empty_like(x)

    log("planning LEM (dense, fp64, decay-bound halo)")
    plan = lem.Plan(opr, p.dt, method="dense", core=16, halo=0, halo_min=4, halo_max=32,
                    halo_tol=args.halo_tol, n_states=ns, autotune=True)
    q = plan.query()
    h = q["halo_max"]
    nloc = (16 + 2 * h) ** 2
    plan.step(x, y, args.warmup)
    torch.cuda.synchronize()
    wall, ev_ms = timed_steps(plan, x, y, args.steps, torch)
    value = N * ns * args.steps / wall
    kern_ms = ev_ms / args.steps
    flops = 2.0 * nloc * N * ns
    achieved = flops / (kern_ms * 1e-3) / 1e12
    log(f"LEM fp64 h={h}: {value:.3e} DOF-steps/s, {kern_ms * 1e3:.1f} us/step, "
        f"{achieved:.1f} TFLOP/s")

    extras = {}
    if not args.no_fp32:  # float32 application of the same blocks
        plan32 = lem.Plan(opr, p.dt, method="dense", precision="fp32", core=16, halo=h,
                          n_states=ns, autotune=True)
        plan32.step(x, y, args.warmup)
        w32, e32 = timed_steps(plan32, x, y, args.steps, torch)
        extras["lem_fp32"] = {"value": N * ns * args.steps / w32,
                              "us_per_step": 1e3 * e32 / args.steps,
                              "tflops": flops / (e32 / args.steps * 1e-3) / 1e12}

    # accuracy against the exact global exponential (global Krylov, tol 1e-13)
    acc = {}
    if not args.no_global:
        log("global Krylov comparator")
        ref_plan = lem.Plan(opr, p.dt, method="global", n_states=ns, krylov_tol=1e-13)
        k = args.acc_steps if args.acc_steps > 0 else 100
        g = torch.empty_like(x)
        ref_plan.step(x, g, k)
        yl = torch.empty_like(x)
        plan.step(x, yl, k)
        torch.cuda.synchronize()
        err = (torch.linalg.norm(yl - g) / torch.linalg.norm(g)).item()
        acc["lem_vs_global_rel_l2"] = err
        acc["acc_steps"] = k
        cfg4 = lem.Plan(opr, p.dt, method="dense", core=16, halo=4, n_states=ns)
        y4 = torch.empty_like(x)
        cfg4.step(x, y4, k)
        torch.cuda.synchronize()
        acc["halo4_vs_global_rel_l2"] = (torch.linalg.norm(y4 - g) / torch.linalg.norm(g)).item()
        # timed global comparator at the same accuracy class (1e-8 per step)
        gplan = lem.Plan(opr, p.dt, method="global", n_states=ns, krylov_tol=1e-8)
        gq = gplan.query()
        gplan.step(x, g, 1)
        gw, gev = timed_steps(gplan, x, g, args.global_steps, torch)
        gval = N * ns * args.global_steps / gw
        extras["global_krylov"] = {"value": gval, "ms_per_step": 1e3 * gw / args.global_steps,
                                   "m": gq["m_max"], "substeps": gq["substeps_max"],
                                   "tol_per_step": 1e-8}
        extras["lem_over_global"] = value / gval
        log(f"global Krylov: {gval:.3e} DOF-steps/s; LEM/global = {value / gval:.1f}x; "
            f"LEM vs global rel l2 after {k} steps = {err:.2e}")

    if args.copy_mb:
        nbytes = args.copy_mb << 20
        a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").uniform_()
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        extras["reference_copy_bytes"] = nbytes
        del a, b

    cpu = None
    if not args.no_cpu:
        boxes = plan.maps()[0]
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(p, boxes, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D periodic advection-diffusion 256x256, velocity (1,0.5), "
                               "nu=1e-3, dt=2dx, 64 smooth states, 16x16 cores, LEM with "
                               "stored local exponentials (fp64 Pade) applied on FP64 MFMA",
                   "grid": [256, 256], "n_states": ns, "core": 16, "halo": h,
                   "halo_rule": f"decay bound {args.halo_tol:g}/step", "n_loc": nloc,
                   "method": "dense", "plan_ms": q["plan_ms"], "squarings": q["squarings"],
                   "tile_config": q["tile_config"]},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": MFMA_FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / MFMA_FP64_PEAK_TFLOPS,
                     "traffic": measured_traffic("c1", q["tile_config"]),
                     "kernel": "apply_mfma_kernel<double>", "flops_per_launch": flops,
                     "us_per_launch": kern_ms * 1e3},
        "cpu_baseline": cpu,
        "accuracy": acc,
        "extras": extras,
    }
    return out


def _rel(a, b, torch):
    return (torch.linalg.norm(a - b) / torch.linalg.norm(b)).item()


def _line(args, workload: dict, value, unit, steps, wall, dtype, extras, roofline=None,
          higher=True):
    return {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": steps,
            "warmup": args.warmup, "ms_per_step": 1e3 * wall / max(steps, 1),
            "higher_is_better": higher, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": workload, "roofline": roofline, "cpu_baseline": None,
            "extras": extras}


def bench_f1(args) -> dict:
    """256^2 x 64 states of du/dt = A u + g with a constant smooth source per
    state: the exponential-Euler update (5) with g_M on every region (dense,
    FP64), against the forced global Krylov step on the same GPU."""
    import torch
    import lem_inputs as L
    import paper_1505_02248_amd as lem
    torch.cuda.init()
    p = L.workload_2d_ensemble()
    ns = p.states.shape[1]
    g = L.source_fields_2d(p.n, ns, seed=9)
    base = lem.Operator.from_problem(p)
    opr = lem.Operator(base.ndim, base.n, base.dx, base.vel, base.nu, base.nu_field, forcing=g)
    N = p.N
    x = torch.from_numpy(p.states.copy()).to("cuda")
    y = torch.empty_like(x)
    log("planning forced LEM (dense, fp64, decay-bound halo)")
    plan = lem.Plan(opr, p.dt, method="dense", core=16, halo=0, halo_min=4, halo_max=32,
                    halo_tol=args.halo_tol, n_states=ns, autotune=True)
    q = plan.query()
    h = q["halo_max"]
    nloc = (16 + 2 * h) ** 2
    plan.step(x, y, args.warmup)
    torch.cuda.synchronize()
    wall, ev_ms = timed_steps(plan, x, y, args.steps, torch)
    value = N * ns * args.steps / wall
    kern_ms = ev_ms / args.steps
    flops = 2.0 * nloc * N * ns
    achieved = flops / (kern_ms * 1e-3) / 1e12
    extras = {}
    if not args.no_global:
        ref_plan = lem.Plan(opr, p.dt, method="global", n_states=ns, krylov_tol=1e-13)
        k = args.acc_steps if args.acc_steps > 0 else 100
        gref = torch.empty_like(x)
        ref_plan.step(x, gref, k)
        yl = torch.empty_like(x)
        plan.step(x, yl, k)
        torch.cuda.synchronize()
        extras["lem_vs_global_rel_l2"] = (torch.linalg.norm(yl - gref) / torch.linalg.norm(gref)).item()
        extras["acc_steps"] = k
        gplan = lem.Plan(opr, p.dt, method="global", n_states=ns, krylov_tol=1e-8)
        gq = gplan.query()
        gplan.step(x, gref, 1)
        gw, _ = timed_steps(gplan, x, gref, args.global_steps, torch)
        gval = N * ns * args.global_steps / gw
        extras["global_krylov"] = {"value": gval, "ms_per_step": 1e3 * gw / args.global_steps,
                                   "m": gq["m_max"], "substeps": gq["substeps_max"]}
        extras["lem_over_global"] = value / gval
    log(f"forced LEM h={h}: {value:.3e} DOF-steps/s, {kern_ms * 1e3:.1f} us/step, "
        f"{achieved:.1f} TFLOP/s; {extras}")
    workload = {"workload": "2D 256x256 periodic advection-diffusion with a constant smooth "
                            "source per state (du/dt = A u + g), velocity (1,0.5), nu=1e-3, "
                            "dt=2dx, 64 states, 16x16 cores, exponential-Euler LEM step with "
                            "stored exp and phi_1 terms (fp64)",
                "grid": [p.n, p.n], "n_states": ns, "core": 16, "halo": h,
                "halo_rule": f"decay bound {args.halo_tol:g}/step", "n_loc": nloc,
                "plan_ms": q["plan_ms"], "tile_config": q["tile_config"]}
    roof = {"bound": "mfma", "achieved": achieved, "peak": MFMA_FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / MFMA_FP64_PEAK_TFLOPS, "traffic": None,
            "kernel": "apply_mfma_kernel<double> (with the forcing term)",
            "flops_per_launch": flops, "us_per_launch": kern_ms * 1e3}
    return _line(args, workload, value, "DOF-steps/s", args.steps, wall, "f64", extras, roof)


def bench_f2(args) -> dict:
    """Viscous Burgers (nu = 0.05) on 400 cells of [0, 10), dt = dx (Courant ~1,
    mu = 2), 256 Gaussian members, T = 5 (200 steps): exponential
    Rosenbrock-Euler LEM with 8 regions of 50 cells and 15-cell buffers, the
    Jacobian and local phi_1 matrices refreshed every 5 steps, against the same
    method on one region (D = 1) on the same GPU."""
    import numpy as np
    import torch
    import lem_inputs as L
    import paper_1505_02248_amd as lem
    torch.cuda.init()
    n, Lx, nu, ns, steps, K = 400, 10.0, 0.05, 256, 200, 5
    dx = Lx / n
    dt = dx
    u0 = L.gaussian_members(n, Lx, ns, seed=11)
    x = torch.from_numpy(u0).to("cuda")
    out = {}
    for label, core, halo in [("lem_d8_b15", 50, 15), ("global_d1", n, 0)]:
        plan = lem.ErePlan(n, dx, nu, dt, n_states=ns, core=core, halo=halo, refresh=K)
        y = torch.empty_like(x)
        plan.step(x, y, K)  # warm-up (one refresh cycle)
        torch.cuda.synchronize()
        plan2 = lem.ErePlan(n, dx, nu, dt, n_states=ns, core=core, halo=halo, refresh=K)
        t0 = time.perf_counter()
        plan2.step(x, y, steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[label] = {"wall_s": wall, "dof_steps_per_s": n * ns * steps / wall, "state": y.clone()}
        log(f"{label}: {n * ns * steps / wall:.3e} DOF-steps/s, {1e3 * wall / steps:.3f} ms/step")
    a, g = out["lem_d8_b15"]["state"], out["global_d1"]["state"]
    err = (torch.linalg.norm(a - g) / torch.linalg.norm(g)).item()
    mass = (g.sum(0) - x.sum(0)).abs().max().item()
    value = out["lem_d8_b15"]["dof_steps_per_s"]
    extras = {"lem_vs_global_rel_l2": err, "global_mass_drift": mass,
              "global_d1": {"dof_steps_per_s": out["global_d1"]["dof_steps_per_s"],
                            "ms_per_step": 1e3 * out["global_d1"]["wall_s"] / steps},
              "lem_over_global": value / out["global_d1"]["dof_steps_per_s"]}
    workload = {"workload": "1D periodic viscous Burgers (nu=0.05) on 400 cells of [0,10), dt=dx, "
                            "256 Gaussian members, 200 steps (T=5); exponential Rosenbrock-Euler LEM, "
                            "8 regions of 50 cells, 15-cell buffers, Jacobian and local phi_1 matrices "
                            "refreshed every 5 steps (fp64)",
                "n": n, "n_states": ns, "core": 50, "halo": 15, "refresh": K}
    return _line(args, workload, value, "DOF-steps/s", steps, out["lem_d8_b15"]["wall_s"], "f64",
                 extras)


def bench_f3(args) -> dict:
    """1D Schroedinger with a harmonic potential (kappa = 10) on 400 points of
    [-5, 5), T = 1, 4096 Gaussian wave packets: LEM with stored complex local
    exponentials (4 regions of 100 points) at the two settings of the paper's
    Schroedinger table, mu = 2 with 20-point buffers and mu = 4 with 25, against
    the global method (D = 1) on the same GPU; the complex blocks are applied
    in real form on FP64 MFMA."""
    import numpy as np
    import torch
    import lem_inputs as L
    import paper_1505_02248_amd as lem
    torch.cuda.init()
    n, Lx, kappa, ns, T = 400, 10.0, 10.0, 4096, 1.0
    dx = Lx / n
    c0 = L.gaussian_wavepackets(n, Lx, kappa, ns, seed=13)
    x = lem.SchrodingerPlan.to_real_form(torch.from_numpy(c0)).to("cuda")
    y = torch.empty_like(x)
    runs = {}
    for mu, B in ((2, 20), (4, 25)):
        dt = 2 * mu * dx * dx
        steps = int(round(T / dt))
        for D, core, halo in ((4, 100, B), (1, n, 0)):
            t0 = time.perf_counter()
            plan = lem.SchrodingerPlan(n, Lx, kappa, dt, n_states=ns, core=core, halo=halo,
                                       autotune=True)
            torch.cuda.synchronize()
            t_plan = time.perf_counter() - t0
            plan.step(x, y, args.warmup)
            torch.cuda.synchronize()
            wall, ev_ms = timed_steps(plan, x, y, steps, torch)
            q = plan.query()
            key = f"mu{mu}_B{B}_D{D}"
            runs[key] = {"dof_steps_per_s": n * ns * steps / wall, "ms_per_step": 1e3 * wall / steps,
                         "us_per_launch": 1e3 * ev_ms / steps, "plan_s": t_plan, "steps": steps,
                         "time_to_solution_s": t_plan + wall, "squarings": q["squarings"],
                         "tile": q["tile_config"], "state": y.clone()}
            log(f"{key}: {runs[key]['dof_steps_per_s']:.3e} DOF-steps/s, "
                f"{runs[key]['us_per_launch']:.1f} us/step, plan {t_plan:.3f} s")
    extras = {}
    for mu, B in ((2, 20), (4, 25)):
        a, g = runs[f"mu{mu}_B{B}_D4"], runs[f"mu{mu}_B{B}_D1"]
        err = (torch.linalg.norm(a["state"] - g["state"]) / torch.linalg.norm(g["state"])).item()
        extras[f"mu{mu}_B{B}"] = {
            "lem_d4": {k: v for k, v in a.items() if k != "state"},
            "global_d1": {k: v for k, v in g.items() if k != "state"},
            "lem_vs_global_rel_l2": err,
            "lem_over_global_steps": a["dof_steps_per_s"] / g["dof_steps_per_s"],
            "lem_over_global_time_to_solution": g["time_to_solution_s"] / a["time_to_solution_s"]}
    head = runs["mu2_B20_D4"]
    rows, cols, nb = 200, 2 * (100 + 2 * 20), 4
    flops = 2.0 * rows * cols * nb * ns
    achieved = flops / (head["us_per_launch"] * 1e-6) / 1e12
    roof = {"bound": "mfma", "achieved": achieved, "peak": MFMA_FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / MFMA_FP64_PEAK_TFLOPS, "traffic": None,
            "kernel": "apply_mfma_kernel<double>", "flops_per_launch": flops,
            "us_per_launch": head["us_per_launch"]}
    workload = {"workload": "1D Schroedinger c_t = (i/2) c_xx - i (kappa/2) x^2 c, kappa=10, 400 "
                            "points of [-5,5), T=1, 4096 Gaussian wave packets; LEM with stored "
                            "complex local exponentials (fp64 Pade, real form), 4 regions of 100 "
                            "points, mu=2 (dt=4dx^2, 400 steps), 20-point buffers",
                "n": n, "n_states": ns, "core": 100, "halo": 20, "mu": 2}
    steps = head["steps"]
    line = _line(args, workload, head["dof_steps_per_s"], "DOF-steps/s", steps,
                 head["ms_per_step"] * steps / 1e3, "f64", extras, roofline=roof)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline_schrodinger(c0[:, :64], Lx, kappa, 4 * dx * dx, 100, 20,
                                                        args.cpu_seconds)
    return line


def cpu_baseline_schrodinger(c0, Lx, kappa, dt, core, halo, budget_s):
    """The oracle's complex LEM steps (numpy) on a sample of members."""
    from oracle import schrodinger as SCH
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    n, k = c0.shape
    t0 = time.perf_counter()
    SCH.lem_blocks(n, Lx, kappa, dt, core, halo)  # local exponentials (excluded below)
    t_blocks = time.perf_counter() - t0
    t0 = time.perf_counter()
    SCH.lem_run(c0, Lx, kappa, dt, 50, core, halo)
    per_step = max((time.perf_counter() - t0 - t_blocks) / 50, 1e-6)
    steps = int(min(4000, max(50, budget_s / per_step)))
    t0 = time.perf_counter()
    SCH.lem_run(c0, Lx, kappa, dt, steps, core, halo)
    el = max(time.perf_counter() - t0 - t_blocks, 1e-9)
    return {"value": n * k * steps / el, "unit": "DOF-steps/s", "cores": int(cores),
            "kind": "oracle", "sample": f"{steps} LEM steps of {k} members (local exponentials "
            f"excluded)"}


def bench_f4(args) -> dict:
    """Variable divergence-free velocity and anisotropic column-wise
    decompositions (eq. ibv2d, section 4.3):
    (A) 512^2 single periodic vortex, Courant 2, nu = 1e-4, 64 Gaussian blobs,
        16^2 cores with decay-bound buffers: LEM with one stored block per region
        (FP64 MFMA), LEM with Krylov local actions (uneven cores), and the global
        Krylov method;
    (B) 128^2 anisotropic mesh (dy = dx/16), horizontal Courant 0.8, vertical
        diffusion number 6, 64 blobs: Krylov LEM on column-wise cores (8 columns
        wide) against square 16^2 cores and the global method."""
    import torch
    import lem_inputs as L
    import paper_1505_02248_amd as lem
    torch.cuda.init()
    stream = torch.cuda.Stream()
    steps = min(args.steps, 40)
    out = {}

    def timed(plan, x, k):
        y = torch.empty_like(x)
        plan.step(x, y, 2, stream=stream)
        stream.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        plan.step(x, y, k, stream=stream)
        e1.record(stream)
        stream.synchronize()
        return (time.perf_counter() - t0) / k, e0.elapsed_time(e1) / k

    def err_vs(plan, ref, x, k):
        y = torch.empty_like(x)
        plan.step(x, y, k, stream=stream)
        stream.synchronize()
        return _rel(y, ref, torch)

    with torch.cuda.stream(stream):
        # (A) vortex
        p = L.workload_2d_vortex(n=512, n_states=64, courant=2.0)
        opr = lem.Operator.from_problem(p)
        ns = p.states.shape[1]
        x = torch.from_numpy(p.states.copy()).to("cuda")
        ref = torch.empty_like(x)
        lem.Plan(opr, p.dt, method="global", n_states=ns, krylov_tol=1e-13, stream=stream).step(
            x, ref, 3, stream=stream)
        log("planning stored blocks per region (vortex, 1024 blocks)")
        t0 = time.perf_counter()
        dplan = lem.Plan(opr, p.dt, method="dense", core=16, halo=0, halo_min=2, halo_max=24,
                         halo_tol=1e-8, n_states=ns, autotune=True, expm="taylor",
                         stream=stream)
        stream.synchronize()
        dplan_s = time.perf_counter() - t0
        dq = dplan.query()
        t_dense, ev_dense = timed(dplan, x, steps)
        err_dense = err_vs(dplan, ref, x, 3)
        log(f"vortex stored-block LEM: {1e3 * t_dense:.3f} ms/step, plan {dplan_s:.1f} s, "
            f"err {err_dense:.2e}")
        kplan = lem.Plan(opr, p.dt, method="krylov", core=0, halo=0, halo_min=2, halo_max=16,
                         halo_tol=1e-8, n_states=ns, krylov_tol=1e-10, use_graph=True,
                         krylov_m_max=args.krylov_m_max, autotune=True, stream=stream)
        kq = kplan.query()
        t_kry, _ = timed(kplan, x, max(3, steps // 8))
        err_kry = err_vs(kplan, ref, x, 3)
        gplan = lem.Plan(opr, p.dt, method="global", n_states=ns, krylov_tol=1e-10, stream=stream)
        gq = gplan.query()
        t_glob, _ = timed(gplan, x, 3)
        log(f"vortex Krylov LEM {1e3 * t_kry:.2f} ms/step, global {1e3 * t_glob:.2f} ms/step")
        nloc = (16 + 2 * dq["halo_max"]) ** 2
        flops = 2.0 * nloc * 256 * ns * dq["n_blocks"]
        out["vortex"] = {
            "stored_blocks": {"ms_per_step": 1e3 * t_dense, "us_per_launch": 1e3 * ev_dense,
                              "plan_s": dplan_s, "halo": dq["halo_max"], "n_blocks": dq["n_blocks"],
                              "bytes_blocks": dq["bytes_blocks"], "tile": dq["tile_config"],
                              "rel_l2_vs_global_after_3_steps": err_dense},
            "krylov_lem": {"ms_per_step": 1e3 * t_kry, "halo_range": [kq["halo_min"], kq["halo_max"]],
                           "m_range": [kq["m_min"], kq["m_max"]], "substeps_max": kq["substeps_max"],
                           "n_blocks": kq["n_blocks"], "n_loc_max": kq["n_loc_max"],
                           "plan_ms": kq["plan_ms"], "rel_l2_vs_global_after_3_steps": err_kry},
            "global": {"ms_per_step": 1e3 * t_glob, "m": gq["m_max"], "substeps": gq["substeps_max"]},
            "stored_over_global_per_step": t_glob / t_dense,
            "krylov_lem_over_global_per_step": t_glob / t_kry,
            "break_even_steps_vs_global": dplan_s / max(t_glob - t_dense, 1e-12)}
        # (B) anisotropic mesh: column-wise against square cores
        pb = L.workload_2d_columns(n=128, n_states=64)
        ob = lem.Operator.from_problem(pb)
        nsb = pb.states.shape[1]
        xb = torch.from_numpy(pb.states.copy()).to("cuda")
        refb = torch.empty_like(xb)
        lem.Plan(ob, pb.dt, method="global", n_states=nsb, krylov_tol=1e-13, stream=stream).step(
            xb, refb, 3, stream=stream)
        res = {}
        for label, kw in (("columns", dict(core=8, columns=True)), ("square", dict(core=16))):
            pl = lem.Plan(ob, pb.dt, method="krylov", halo=0, halo_min=2, halo_max=24,
                          halo_tol=1e-8, n_states=nsb, krylov_tol=1e-10, use_graph=True,
                          krylov_m_max=args.krylov_m_max, stream=stream, **kw)
            qb = pl.query()
            t, _ = timed(pl, xb, steps)
            res[label] = {"dof_steps_per_s": pb.N * nsb / t, "ms_per_step": 1e3 * t,
                          "rel_l2_vs_global_after_3_steps": err_vs(pl, refb, xb, 3),
                          "n_blocks": qb["n_blocks"], "halo_range": [qb["halo_min"], qb["halo_max"]],
                          "halo_clamped_blocks": qb["halo_clamped"], "n_loc_max": qb["n_loc_max"],
                          "m_range": [qb["m_min"], qb["m_max"]],
                          "substeps_max": qb["substeps_max"]}
            log(f"anisotropic {label}: {res[label]}")
        gb = lem.Plan(ob, pb.dt, method="global", n_states=nsb, krylov_tol=1e-10, stream=stream)
        tg, _ = timed(gb, xb, 3)
        res["global"] = {"dof_steps_per_s": pb.N * nsb / tg, "ms_per_step": 1e3 * tg,
                         "m": gb.query()["m_max"], "substeps": gb.query()["substeps_max"]}
        out["anisotropic_columns"] = res
    achieved = flops / (ev_dense * 1e-3) / 1e12
    roof = {"bound": "mfma", "achieved": achieved, "peak": MFMA_FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / MFMA_FP64_PEAK_TFLOPS, "traffic": None,
            "kernel": "apply_mfma_kernel<double> (one stored block per region)",
            "flops_per_launch": flops, "us_per_launch": 1e3 * ev_dense}
    wl = {"workload": "2D 512x512 periodic advection-diffusion -div(a c) + nu lap c, single "
                      "divergence-free vortex (face velocities from a stream function), Courant 2, "
                      "nu=1e-4, 64 Gaussian blobs; LEM with one stored FP64 block per 16^2 core "
                      "(1024 blocks, buffers from the decay bound at 1e-8/step, exponentials by "
                      "the GEMM-only Taylor pipeline), FP64 MFMA apply",
          "n": 512, "n_states": 64, "core": 16, "halo": dq["halo_max"]}
    value = p.N * ns / t_dense
    return _line(args, wl, value, "DOF-steps/s", steps, t_dense * steps, "f64", out, roofline=roof)


def bench_c0(args) -> dict:
    """1D periodic advection-diffusion, N = 1024, 16 cores of 64 points, 100 steps."""
    import torch
    import lem_inputs as L
    import paper_1505_02248_amd as lem
    p = L.workload_1d()
    opr = lem.Operator.from_problem(p)
    x = torch.from_numpy(p.states.copy()).to("cuda")
    steps = 100
    ref = torch.empty_like(x)
    lem.Plan(opr, p.dt, method="global", krylov_tol=1e-14).step(x, ref, steps)
    res = {}
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for label, kw in [("lem_krylov_bound", dict(method="krylov", halo=0)),
                          ("lem_dense_bound", dict(method="dense", halo=0)),
                          ("lem_krylov_h16", dict(method="krylov", halo=16)),
                          ("lem_dense_h16", dict(method="dense", halo=16)),
                          ("global_krylov", dict(method="global"))]:
            plan = lem.Plan(opr, p.dt, core=64, halo_min=4, halo_max=64,
                            halo_tol=args.halo_tol, krylov_tol=1e-10, use_graph=True,
                            stream=stream, **kw)
            y = torch.empty_like(x)
            plan.step(x, y, 3, stream=stream)
            stream.synchronize()
            t0 = time.perf_counter()
            plan.step(x, y, steps, stream=stream)
            stream.synchronize()
            wall = time.perf_counter() - t0
            q = plan.query()
            res[label] = {"dof_steps_per_s": p.N * steps / wall, "us_per_step": 1e6 * wall / steps,
                          "rel_l2_vs_global_exact": _rel(y, ref, torch), "halo": q["halo_max"],
                          "m": q["m_max"], "substeps": q["substeps_max"]}
            log(label, res[label])
            res[label]["_plan"] = plan
    best = max(("lem_krylov_bound", "lem_dense_bound"), key=lambda k: res[k]["dof_steps_per_s"])
    bplan = res[best]["_plan"]
    bq = bplan.query()
    boxes = bplan.maps()[0]
    # algorithmic bytes of one step of the best form: the Krylov basis traffic
    # (|M| 8 (m(m+1)+3m) nsub per region) or, for stored blocks, the one
    # stored core block, the gathered regions and the written cores
    us = res[best]["us_per_step"]
    if best == "lem_krylov_bound":
        step_bytes = float(bq["krylov_bytes_step"])
        achieved = step_bytes / (us * 1e-6) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "kernel": f"{best} (whole step; latency bound: 16 regions of 64 points fill 16 "
                          "of 256 compute units)",
                "bytes_per_step": step_bytes, "us_per_step": us}
    else:
        # one stored block, 16 regions: 2 x 64 rows x |M| columns per region;
        # with resident steps one workgroup (one CU) runs all 100 steps
        nloc = 64 + 2 * res[best]["halo"]
        flops = 2.0 * 64 * nloc * len(boxes)
        achieved = flops / (us * 1e-6) / 1e12
        resident = bq.get("resident_steps", 0) == 1
        roof = {"bound": "mfma", "achieved": achieved, "peak": MFMA_FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / MFMA_FP64_PEAK_TFLOPS, "traffic": None,
                "kernel": ("dense_resident_kernel (all 100 steps in one launch on one CU: states "
                           "in LDS, stored-block rows in registers; bound by the per-step MFMA "
                           "chain, not by the chip's peak)") if resident else
                          f"{best} (whole step, one graph replay; launch-latency bound)",
                "flops_per_step": flops, "us_per_step": us,
                "frac_of_one_cu": achieved / (MFMA_FP64_PEAK_TFLOPS / 256)}
    for r in res.values():
        r.pop("_plan", None)
    wl = {"workload": "1D periodic advection-diffusion N=1024, a=1, nu=1e-3, dt=4dx, "
                      "16 cores of 64 points, 100 steps per call, FP64 (dense: all steps in "
                      "one launch; Krylov: HIP graph per step)",
          "best_lem": best, "resident_steps": int(bq.get("resident_steps", 0))}
    line = _line(args, wl, res[best]["dof_steps_per_s"], "DOF-steps/s", steps,
                 res[best]["us_per_step"] * steps * 1e-6, "f64",
                 dict(res, lem_over_global=res[best]["dof_steps_per_s"] /
                      res["global_krylov"]["dof_steps_per_s"]), roofline=roof)
    if not args.no_cpu:
        log("cpu baseline (oracle, all 16 regions)")
        kw = ({"krylov_above": 1, "krylov_m": 40, "krylov_tol": 1e-10}
              if best == "lem_krylov_bound" else {})
        line["cpu_baseline"] = cpu_baseline(p, boxes, min(args.cpu_seconds, 10.0), **kw)
    return line


def bench_c2(args) -> dict:
    """2D 1024^2 lognormal nu, uneven cores (16/32/64 per 64^2 tile), decay-bound
    halos, calibrated Krylov dimensions up to 40, one HIP graph per step."""
    import torch
    import lem_inputs as L
    import paper_1505_02248_amd as lem
    p = L.workload_2d_variable()
    opr = lem.Operator.from_problem(p)
    x = torch.from_numpy(p.states.copy()).to("cuda")
    stream = torch.cuda.Stream()
    steps = min(args.steps, 50)
    with torch.cuda.stream(stream):
        log("planning uneven Krylov LEM (1024^2)")
        t0 = time.perf_counter()
        plan = lem.Plan(opr, p.dt, method="krylov", core=0, halo=0, halo_min=4, halo_max=16,
                        halo_tol=1e-8, krylov_m_max=args.krylov_m_max, krylov_tol=1e-10,
                        use_graph=True, autotune=True, stream=stream)
        plan_s = time.perf_counter() - t0
        q = plan.query()
        boxes = plan.maps()[0]
        m_blk, sub_blk = plan.krylov()
        y = torch.empty_like(x)
        plan.step(x, y, 2, stream=stream)
        stream.synchronize()
        log(f"timing {steps} steps")
        wall, ev = _time_stream(plan, x, y, steps, stream, torch)
        q = plan.query()
        lem_val = p.N * steps / wall
        step_s = ev * 1e-3 / steps
        log(f"LEM: {lem_val:.3e} DOF-steps/s, {1e3 * step_s:.2f} ms/step")
        # accuracy and the global comparator
        acc_steps = 3
        ref = torch.empty_like(x)
        lem.Plan(opr, p.dt, method="global", krylov_tol=1e-13, stream=stream).step(
            x, ref, acc_steps, stream=stream)
        ya = torch.empty_like(x)
        plan.step(x, ya, acc_steps, stream=stream)
        stream.synchronize()
        err = _rel(ya, ref, torch)
        gplan = lem.Plan(opr, p.dt, method="global", krylov_tol=1e-10, stream=stream)
        gq = gplan.query()
        g = torch.empty_like(x)
        gplan.step(x, g, 1, stream=stream)
        stream.synchronize()
        gw, _ = _time_stream(gplan, x, g, 3, stream, torch)
        gwall = gw / 3
        # the partitions the autotuner weighs, each planned alone: largest core
        # 32 or 64 points, Krylov dimension capped at 30 or at krylov_m_max
        cands = {}
        for cmax, mcap in ((32, 30), (64, 30), (32, args.krylov_m_max), (64, args.krylov_m_max)):
            key = f"core_max{cmax}_m{mcap}"
            if key in cands:
                continue
            cp = lem.Plan(opr, p.dt, method="krylov", core=0, halo=0, halo_min=4, halo_max=16,
                          halo_tol=1e-8, krylov_m_max=mcap, krylov_tol=1e-10, use_graph=True,
                          core_max=cmax, stream=stream)
            cy = torch.empty_like(x)
            cp.step(x, cy, 2, stream=stream)
            _, cev = _time_stream(cp, x, cy, 10, stream, torch)
            cp.step(x, cy, acc_steps, stream=stream)
            stream.synchronize()
            cq = cp.query()
            cb = cp.maps()[0]
            cands[key] = {"ms_per_step": cev / 10, "n_blocks": cq["n_blocks"],
                          "cores": {int(c): int((cb[:, 2] == c).sum()) for c in np.unique(cb[:, 2])},
                          "m_range": [cq["m_min"], cq["m_max"]], "n_loc_max": cq["n_loc_max"],
                          "rel_l2_vs_global_after_3_steps": _rel(cy, ref, torch)}
            log(key, cands[key])
            del cp
    cores = {int(c): int((boxes[:, 2] == c).sum()) for c in np.unique(boxes[:, 2])}
    wl = {"workload": "2D 1024x1024 periodic diffusion-advection, lognormal nu (median 1e-3, "
                      "sigma_log 1), velocity (1,0), dt=dx/4, uneven cores 16-64 per 64^2 tile, "
                      "decay-bound halos 4-16 (1e-8/step), calibrated Krylov m per block, "
                      "HIP graph per step, FP64",
          "n_blocks": q["n_blocks"], "cores": cores, "halo_range": [q["halo_min"], q["halo_max"]],
          "halo_clamped_blocks": q["halo_clamped"], "m_range": [q["m_min"], q["m_max"]],
          "substeps_max": q["substeps_max"], "n_loc_max": q["n_loc_max"], "plan_s": plan_s}
    extras = {"lem_rel_l2_vs_global_after_3_steps": err, "max_estimate": q["max_estimate"],
              "device_status": q["device_status"],
              "krylov_bytes_step": q["krylov_bytes_step"],
              "krylov_bytes_streamed": q["krylov_bytes_streamed"],
              "m_histogram": {int(k): int((m_blk == k).sum()) for k in np.unique(m_blk)},
              "global_krylov": {"dof_steps_per_s": p.N / gwall, "ms_per_step": 1e3 * gwall,
                                "m": gq["m_max"], "substeps": gq["substeps_max"]},
              "lem_over_global": lem_val / (p.N / gwall),
              "partition_candidates": cands}
    log(extras)
    # every launch of the step overlaps (forked buckets): the algorithmic basis
    # traffic of the whole step over the step's event time bounds the rate of
    # the streaming kernels from below
    achieved = q["krylov_bytes_step"] / step_s / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": "Krylov LEM step (all buckets; algorithmic |M| 8 (m(m+1)+3m) nsub B per "
                      "block and member)",
            "bytes_per_step": q["krylov_bytes_step"], "us_per_step": step_s * 1e6}
    line = _line(args, wl, lem_val, "DOF-steps/s", steps, wall, "f64", extras, roofline=roof)
    if not args.no_cpu:
        log("cpu baseline (oracle, sampled regions)")
        bx = boxes[np.argsort(-boxes[:, 2], kind="stable")]  # largest cores first
        pick = np.concatenate([bx[bx[:, 2] == c][:2] for c in sorted(cores, reverse=True)])
        line["cpu_baseline"] = cpu_baseline(p, pick, args.cpu_seconds, sample_blocks=len(pick),
                                            krylov_above=1, krylov_m=40, krylov_tol=1e-10)
    return line


def _time_stream(plan, x, y, k, stream, torch):
    """k steps of plan as one lem_step on `stream`, bracketed by HIP events on
    that stream: (wall s, event ms)."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    plan.step(x, y, k, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, e0.elapsed_time(e1)


def bench_c3(args) -> dict:
    """512^2 x 128 states, 32^2 cores: stored FP64 Pade blocks applied on FP64
    MFMA with the decay-bound buffer (the headline), against the global Krylov
    method on the same grid; FP32 and split-bf16 arms of the same blocks, the
    configured 8-point buffer and the 256^2 x 64-state workload as extras."""
    import torch
    import lem_inputs as L
    import paper_1505_02248_amd as lem
    torch.cuda.init()
    p = L.workload_2d_mixed()  # 512^2, 128 smooth states
    opr = lem.Operator.from_problem(p)
    ns = p.states.shape[1]
    N = p.N
    x = torch.from_numpy(p.states.copy()).to("cuda")
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    arms = [a for a in args.arms.split(",") if a]

    log("planning LEM (dense, fp64, 32^2 cores, decay-bound halo)")
    plan = lem.Plan(opr, p.dt, method="dense", core=32, halo=0, halo_min=4, halo_max=32,
                    halo_tol=args.halo_tol, n_states=ns, autotune=True)
    q = plan.query()
    h = q["halo_max"]
    nloc = (32 + 2 * h) ** 2
    plan.step(x, y, args.warmup)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps (h={h}, tile {q['tile_config']})")
    wall, ev_ms = _time_stream(plan, x, y, args.steps, stream, torch)
    value = N * ns * args.steps / wall
    kern_ms = ev_ms / args.steps
    flops = 2.0 * 1024 * nloc * 256 * ns  # core rows x local columns x blocks x states
    achieved = flops / (kern_ms * 1e-3) / 1e12
    log(f"LEM fp64 h={h}: {value:.3e} DOF-steps/s, {kern_ms * 1e3:.1f} us/step, "
        f"{achieved:.1f} TFLOP/s ({achieved / MFMA_FP64_PEAK_TFLOPS:.1%} of FP64 MFMA peak)")

    extras = {}
    peaks = {"fp64": MFMA_FP64_PEAK_TFLOPS, "fp32": MFMA_FP32_PEAK_TFLOPS,
             "bf16x3": MFMA_BF16_PEAK_TFLOPS, "bf16x2": MFMA_BF16_PEAK_TFLOPS}
    terms = {"fp64": 1, "fp32": 1, "bf16x3": 6, "bf16x2": 3}
    y64 = torch.empty_like(x)
    plan.step(x, y64, 1)
    for prec in arms:  # the same blocks applied in reduced precision
        log(f"planning the {prec} arm")
        pl = lem.Plan(opr, p.dt, method="dense", precision=prec, core=32, halo=h, n_states=ns,
                      autotune=True)
        pl.step(x, y, args.warmup)
        w, e = _time_stream(pl, x, y, args.steps, stream, torch)
        yp = torch.empty_like(x)
        pl.step(x, yp, 1)
        us = 1e3 * e / args.steps
        extras[f"lem_{prec}"] = {
            "value": N * ns * args.steps / w, "us_per_step": us,
            "rel_l2_vs_fp64_one_step": _rel(yp, y64, torch),
            "tflops_algorithmic": flops / us / 1e6,
            "mfma_frac": flops * terms[prec] / us / 1e6 / peaks[prec],
            "tile_config": pl.query()["tile_config"]}
        log(f"{prec}: {extras[f'lem_{prec}']}")
        del pl

    if args.kron:
        # the same local exponentials in Kronecker-factored form (the box
        # matrix of a constant-coefficient operator is a Kronecker sum):
        # two contractions of 2 L^2 c + 2 L c^2 flops per block and member
        log("planning the Kronecker-factored arm")
        kp = lem.Plan(opr, p.dt, method="kronecker", core=32, halo=h, n_states=ns)
        kp.step(x, y, args.warmup)
        wk, ek = _time_stream(kp, x, y, args.steps, stream, torch)
        yk = torch.empty_like(x)
        kp.step(x, yk, 1)
        side = 32 + 2 * h
        kflops = (2.0 * side * side * 32 + 2.0 * side * 32 * 32) * 256 * ns
        kus = 1e3 * ek / args.steps
        extras["lem_kronecker_fp64"] = {
            "value": N * ns * args.steps / wk, "us_per_step": kus,
            "rel_l2_vs_dense_fp64_one_step": _rel(yk, y64, torch),
            "flops_per_step": kflops, "tflops": kflops / kus / 1e6,
            "mfma_frac": kflops / kus / 1e6 / MFMA_FP64_PEAK_TFLOPS,
            "gbs_state": 2.0 * N * ns * 8 / kus / 1e3,
            "plan_ms": kp.query()["plan_ms"]}
        log(f"kronecker: {extras['lem_kronecker_fp64']}")
        del kp

    acc = {}
    if not args.no_global:
        k = args.acc_steps if args.acc_steps > 0 else args.steps
        log(f"global Krylov reference (tol 1e-13), {k} steps")
        ref_plan = lem.Plan(opr, p.dt, method="global", n_states=ns, krylov_tol=1e-13)
        g = torch.empty_like(x)
        ref_plan.step(x, g, k)
        yl = torch.empty_like(x)
        plan.step(x, yl, k)
        torch.cuda.synchronize()
        acc["lem_vs_global_rel_l2"] = _rel(yl, g, torch)
        acc["acc_steps"] = k
        del ref_plan
        log("LEM at the configured 8-point buffer")
        cfg8 = lem.Plan(opr, p.dt, method="dense", core=32, halo=8, n_states=ns, autotune=True)
        y8 = torch.empty_like(x)
        cfg8.step(x, y8, k)
        torch.cuda.synchronize()
        acc["halo8_vs_global_rel_l2"] = _rel(y8, g, torch)
        w8, e8 = _time_stream(cfg8, x, y8, args.steps, stream, torch)
        extras["lem_fp64_halo8"] = {"value": N * ns * args.steps / w8,
                                    "us_per_step": 1e3 * e8 / args.steps}
        del cfg8, y8
        log("global Krylov comparator (tol 1e-8 per step)")
        gplan = lem.Plan(opr, p.dt, method="global", n_states=ns, krylov_tol=1e-8)
        gq = gplan.query()
        gk = torch.empty_like(x)
        gplan.step(x, gk, k)
        torch.cuda.synchronize()
        acc["global_1e-8_vs_global_1e-13_rel_l2"] = _rel(gk, g, torch)
        gplan.step(x, gk, 1)
        gw, _ = _time_stream(gplan, x, gk, args.global_steps, stream, torch)
        gval = N * ns * args.global_steps / gw
        extras["global_krylov"] = {"value": gval, "ms_per_step": 1e3 * gw / args.global_steps,
                                   "m": gq["m_max"], "substeps": gq["substeps_max"],
                                   "tol_per_step": 1e-8}
        extras["lem_over_global"] = value / gval
        log(f"global Krylov: {gval:.3e} DOF-steps/s; LEM/global = {value / gval:.1f}x; "
            f"LEM vs global after {k} steps = {acc['lem_vs_global_rel_l2']:.2e}")
        del gplan, g, gk, yl

    if args.with_c1:
        extras["c1_256x256x64"] = _c1_summary(args, torch, lem, L)

    if args.copy_mb:
        nbytes = args.copy_mb << 20
        a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").uniform_()
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        extras["reference_copy_bytes"] = nbytes
        del a, b

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(p, plan.maps()[0], args.cpu_seconds, sample_blocks=8)

    return {
        "metric": METRIC,
        "value": value,
        "unit": "DOF-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D periodic advection-diffusion 512x512, velocity (1,0.5), "
                               "nu=1e-3, dt=2dx, 128 smooth states, 32x32 cores, LEM with "
                               "stored local exponentials (fp64 Pade) applied on FP64 MFMA",
                   "grid": [512, 512], "n_states": ns, "core": 32, "halo": h,
                   "halo_rule": f"decay bound {args.halo_tol:g}/step", "n_loc": nloc,
                   "method": "dense", "plan_ms": q["plan_ms"], "squarings": q["squarings"],
                   "tile_config": q["tile_config"]},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": MFMA_FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / MFMA_FP64_PEAK_TFLOPS,
                     "traffic": measured_traffic("c3", q["tile_config"]),
                     "kernel": "apply_mfma_kernel<double>", "flops_per_launch": flops,
                     "us_per_launch": kern_ms * 1e3},
        "cpu_baseline": cpu,
        "accuracy": acc,
        "extras": extras,
    }


def _c1_summary(args, torch, lem, L) -> dict:
    """256^2 x 64 states, 16^2 cores, decay-bound buffer: FP64 apply rate and
    its error against the global Krylov action after the same steps."""
    p = L.workload_2d_ensemble()
    opr = lem.Operator.from_problem(p)
    ns = p.states.shape[1]
    x = torch.from_numpy(p.states.copy()).to("cuda")
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    plan = lem.Plan(opr, p.dt, method="dense", core=16, halo=0, halo_min=4, halo_max=32,
                    halo_tol=args.halo_tol, n_states=ns, autotune=True)
    q = plan.query()
    h = q["halo_max"]
    plan.step(x, y, args.warmup)
    w, e = _time_stream(plan, x, y, args.steps, stream, torch)
    flops = 2.0 * 256 * (16 + 2 * h) ** 2 * 256 * ns
    us = 1e3 * e / args.steps
    out = {"value": p.N * ns * args.steps / w, "us_per_step": us, "halo": h,
           "tile_config": q["tile_config"], "mfma_frac": flops / us / 1e6 / MFMA_FP64_PEAK_TFLOPS}
    if not args.no_global:
        ref = lem.Plan(opr, p.dt, method="global", n_states=ns, krylov_tol=1e-13)
        g = torch.empty_like(x)
        ref.step(x, g, args.steps)
        plan.step(x, y, args.steps)
        torch.cuda.synchronize()
        out["lem_vs_global_rel_l2"] = _rel(y, g, torch)
    log(f"c1: {out}")
    return out


def bench_c4(args) -> dict:
    """Served Poisson stream of independent 2D problems (continuous batching):
    --warm-requests requests, then --requests measured ones, arriving in real
    time at 200 req/s; latency and throughput over the measured requests."""
    import numpy as np
    import lem_inputs as L
    import paper_1505_02248_amd as lem
    nw, nm = args.warm_requests, args.requests
    log(f"generating {nw + nm} requests")
    reqs = L.serving_stream(nw + nm)
    import torch
    free, total = torch.cuda.mem_get_info()
    budget = min(32 << 30, int(free * 0.5))
    log(f"device memory free {free / 2**30:.1f} GiB of {total / 2**30:.1f} GiB; "
        f"pool {budget / 2**30:.1f} GiB")
    srv = lem.Server(hbm_budget=budget, max_active=512, krylov_tol=1e-10,
                     krylov_m_max=args.krylov_m_max, max_overhead=args.max_overhead,
                     steps_per_tick=args.steps_per_tick)
    pending = list(reqs)
    ids, done_t, arrival = {}, {}, {}
    t0 = time.perf_counter()
    ticks = 0
    last_log = t0
    while pending or len(done_t) < len(reqs):
        now = time.perf_counter() - t0
        while pending and pending[0].arrival <= now:
            r = pending.pop(0)
            rid = srv.submit(lem.Operator.from_problem(r.problem), r.problem.dt, r.n_steps,
                             r.problem.states[:, 0])
            ids[rid] = r
            arrival[rid] = r.arrival
        active, queued = srv.tick()
        ticks += 1
        now = time.perf_counter() - t0
        for rid in list(ids):
            if rid not in done_t and srv.poll(rid) in ("done", "failed"):
                done_t[rid] = now
        if time.perf_counter() - last_log > 20:
            last_log = time.perf_counter()
            log(f"t={now:.1f}s done {len(done_t)}/{len(reqs)} active {active} queued {queued}")
        if active == 0 and queued == 0 and pending and len(done_t) == len(ids):
            time.sleep(max(0.0, pending[0].arrival - (time.perf_counter() - t0)))
    measured = [rid for rid in ids if ids[rid].rid >= nw]
    lat = np.array([done_t[r] - arrival[r] for r in measured])
    first = min(arrival[r] for r in measured)
    end = max(done_t[r] for r in measured)
    dof = sum(ids[r].problem.N * ids[r].n_steps for r in measured)
    val = dof / (end - first)
    span = max(arrival[r] for r in measured) - first
    offered = dof / span
    methods = {}
    failed = []
    for rid in measured:
        info = srv.request_info(rid)
        methods[info["method"]] = methods.get(info["method"], 0) + 1
        if info["state"] == "failed":
            pr = ids[rid].problem
            failed.append({"n": pr.n, "nu": pr.nu, "dt_over_dx": round(pr.dt / pr.dx),
                           "steps": ids[rid].n_steps, "method": info["method"],
                           "error": info["error"], "steps_done": info["steps_done"],
                           "m_max": info["m_max"], "substeps": info["substeps_max"]})
    wl = {"workload": f"served Poisson stream ({nw} warm-up + {nm} measured requests, 200 req/s) "
                      "of 2D periodic advection-diffusion, n in {64,128,256,512}, nu log-uniform "
                      "[1e-4,1e-2], dt in {1,2,4} dx, 20-200 steps, FP64, continuous batching",
          "requests": nm, "warm_requests": nw, "methods": methods, "pool_bytes": budget,
          "max_overhead": args.max_overhead, "steps_per_tick": args.steps_per_tick,
          "krylov_m_max": args.krylov_m_max}
    extras = {"p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
              "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
              "mean_latency_ms": float(lat.mean() * 1e3), "measured_span_s": end - first,
              "offered_dof_steps_per_s": offered, "ticks": ticks, "failed": len(failed),
              "failed_requests": failed[:20],
              "device_status": srv.query()["device_status"]}
    if args.saturate:
        # capacity: the measured requests all submitted at once (closed loop)
        log(f"saturated: {nm} requests submitted at once")
        sat_ids = {}
        t0 = time.perf_counter()
        for r in reqs[nw:]:
            rid = srv.submit(lem.Operator.from_problem(r.problem), r.problem.dt, r.n_steps,
                             r.problem.states[:, 0])
            sat_ids[rid] = r
        sat_done = {}
        sat_ticks = 0
        while len(sat_done) < len(sat_ids):
            srv.tick()
            sat_ticks += 1
            now = time.perf_counter() - t0
            for rid in sat_ids:
                if rid not in sat_done and srv.poll(rid) in ("done", "failed"):
                    sat_done[rid] = now
        span_s = max(sat_done.values())
        sat_lat = np.array(list(sat_done.values()))
        extras["saturated"] = {
            "dof_steps_per_s": dof / span_s, "seconds": span_s, "ticks": sat_ticks,
            "p50_completion_ms": float(np.percentile(sat_lat, 50) * 1e3),
            "p99_completion_ms": float(np.percentile(sat_lat, 99) * 1e3),
            "failed": sum(srv.poll(r) == "failed" for r in sat_ids)}
    log(extras)
    # algorithmic state traffic of the served steps: every local method reads
    # its boxes ((L/c)^2 values per core point) and writes its cores; the
    # global method reads and writes the state at least once per step
    byts = 0.0
    for rid in measured:
        info, pr = srv.request_info(rid), ids[rid].problem
        ratio = (((info["core"] + 2 * info["halo"]) / info["core"]) ** 2
                 if info["core"] else 1.0)
        byts += 8.0 * pr.N * info["steps_done"] * (ratio + 1.0)
    achieved = byts / (end - first) / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": "all served steps (state read per box + core write per step) over the "
                      "measured span; arrival-rate bound, not a kernel's own rate",
            "bytes": byts}
    line = _line(args, wl, val, "DOF-steps/s", ticks, end - first, "f64", extras, roofline=roof)
    if not args.no_cpu:
        log("cpu baseline (oracle, sampled regions of the measured requests)")
        line["cpu_baseline"] = cpu_baseline_serving(
            [(ids[r].problem, srv.request_info(r)) for r in measured], min(args.cpu_seconds, 20.0))
    return line


def cpu_baseline_serving(reqs, budget_s: float, regions_per_request: int = 4):
    """The oracle on the served requests in arrival order, one step each: for
    a local method the first regions_per_request regions of its partition
    (Krylov action per region, from the initial state), for the global method
    the exact step of the whole grid by FFT, until ~budget_s."""
    from oracle import globalexp as ge
    from oracle import lem as olem
    from oracle import operator as op
    from oracle import partition as P
    cores, model, ncpu = host_cpu()
    done, k, t0 = 0, 0, time.perf_counter()
    sizes = {}
    for pr, info in reqs:
        W = op.from_problem(pr)
        u = pr.states[:, 0]
        if info["core"]:
            bx = P.uniform_boxes(2, pr.n, info["core"], info["halo"])[:regions_per_request]
            olem.step(op.sparse(W), bx, 2, pr.n, u, krylov_above=1, krylov_m=40,
                      krylov_tol=1e-10)
            done += len(bx) * info["core"] ** 2
        else:
            ge.fft_steps(W, u, 1)
            done += pr.N
        k += 1
        sizes[pr.n] = sizes.get(pr.n, 0) + 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "DOF-steps/s", "cores": cores, "kind": "oracle",
            "cpu_model": model, "logical_cpus": ncpu,
            "sample": f"one step of the first {k} measured requests (grid sides {sizes}): "
                      f"{regions_per_request} regions each by the oracle's Krylov action "
                      "(numpy float64), or the whole grid by FFT for global-method requests",
            "seconds": round(el, 3)}


if __name__ == "__main__":
    sys.exit(main())
