#!/usr/bin/env python3
"""NMPC re-solve benchmark on one MI355X.

Workload (default): distillation column, 40 trays (42 states) + reflux and
boilup, horizon 100 implicit-Euler stages of 0.05, alpha ~ U(2,3) from the
seed, sinusoidal feed-composition disturbance, warm-started receding-horizon
re-solves with one symbolic analysis.  A step is one warm re-solve: parameter
upload, every interior-point iteration on the GPU (eval, assembly, supernodal
Cholesky, solves, line search), and the download of u_1 and x_1 for the plant.
The first solve (analyze + cold start) is reported on its own.

Prints one JSON line.  --gpus N with N > 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBPS = 8000.0


TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "factor_distill_medium_hbm_traffic.txt")


def measured_traffic():
    """HBM bytes per factorization from the committed counter summary, or None
    when the factorization kernels changed since the counters were taken."""
    import hashlib
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
        src = os.path.join(os.path.dirname(TRAFFIC_FILE), "..", kv["source_file"])
        if hashlib.sha256(open(src, "rb").read()).hexdigest() != kv["source_sha256"]:
            return None
        return float(kv["bytes_per_factorization"])
    except (OSError, KeyError, ValueError):
        return None


def _percentile(v, q):
    return float(np.percentile(np.asarray(v, dtype=float), q)) if len(v) else float("nan")


def cpu_baseline(seed: int, budget_s: float):
    """The oracle's interior-point method on the host, bounded sample of the
    same workload: one cold solve (untimed set-up), then warm re-solves until
    the time budget is spent."""
    from oracle.distillation import DistillationOCP
    from oracle.ipm import LiftedIPM
    from workloads import distillation_workload
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    w = distillation_workload("medium", seed)
    m = DistillationOCP.from_workload(w)
    ipm = LiftedIPM(m)
    x0, u_prev = w.x0.copy(), w.u_prev0.copy()
    m.set_parameters(x0=x0, zF=w.zF(0), u_prev=u_prev)
    res = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
    times, iters = [], 0
    t_start = time.perf_counter()
    r = 0
    while time.perf_counter() - t_start < budget_s and r < w.n_resolves:
        x0 = w.next_measurement(m.x1(res.state.y), r)
        u_prev = m.u1(res.state.y)
        m.set_parameters(x0=x0, zF=w.zF(r + 1), u_prev=u_prev)
        t = time.perf_counter()
        res = ipm.solve(res.state, ipm.o.mu0_warm)
        times.append(time.perf_counter() - t)
        iters += res.iters
        r += 1
    tot = sum(times)
    return {"value": iters / tot if tot > 0 else None, "unit": "IPM iters/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"medium distillation seed {seed}: {len(times)} warm re-solves after one cold solve "
                      f"({iters} IPM iterations, {tot:.1f} s)",
            "p50_resolve_ms": _percentile([t * 1e3 for t in times], 50)}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES, 10 times (counter calibration)")
    a = ap.parse_args(argv)
    if a.copy_calibration:
        import torch
        n = a.copy_calibration // 8
        src = torch.arange(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 8, "copies": 10}), flush=True)
        return 0
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build measures one GPU only; multi-GPU runs are not supported", file=sys.stderr)
        return 2

    import torch
    from paper_2606_04725_amd import nmpc as N
    from workloads import distillation_workload

    if not torch.cuda.is_available() or not N.device_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    w = distillation_workload("medium", a.seed, n_resolves=a.warmup + a.steps + 1)
    p = N.Problem(N.distillation_structure(w.N, w.H, w.dt, w.alpha, F=w.F, rho=w.rho))
    sp = [w.xD_sp, w.xB_sp]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.analyze()
    t_an = time.perf_counter() - t0
    p.set_parameters(w.x0, setpoint=sp, traj=w.zF(0), u_prev=w.u_prev0)
    r0 = p.solve(warm=False)
    sol = p.solution()
    t_first = time.perf_counter() - t0
    if r0.status != 0:
        print(f"bench.py: cold solve failed with status {r0.status}", file=sys.stderr)
        return 1
    sym = p.symbolic_sizes()
    opts = N.default_options(timing=1)

    def resolve(k):
        nonlocal sol
        x0 = w.next_measurement(sol["x1"], k)
        t = time.perf_counter()
        p.set_parameters(x0, setpoint=sp, traj=w.zF(k + 1), u_prev=sol["u1"])
        res = p.solve(warm=True, options=opts)
        sol = p.solution()
        return res, time.perf_counter() - t

    for k in range(a.warmup):
        res, _ = resolve(k)
        if res.status != 0:
            print(f"bench.py: warm-up re-solve {k} returned status {res.status}", file=sys.stderr)
            return 1
    torch.cuda.synchronize()
    t_begin = time.perf_counter()
    lat, iters, facts, ms_fact, statuses = [], 0, 0, 0.0, []
    phase = dict(eval=0.0, assemble=0.0, factor=0.0, solve=0.0, linesearch=0.0)
    for k in range(a.warmup, a.warmup + a.steps):
        res, dt = resolve(k)
        lat.append(dt * 1e3)
        iters += res.iters
        facts += res.factorizations
        ms_fact += res.ms_factor
        statuses.append(res.status)
        for key in phase:
            phase[key] += getattr(res, "ms_" + key)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_begin
    nk = int(p.nnz_k)
    bytes_per_factor = 8.0 * (nk + sym["nnz_l"])
    achieved = (facts * bytes_per_factor / (ms_fact * 1e-3)) / 1e9 if ms_fact > 0 else None
    gflops = (facts * sym["flops"] / (ms_fact * 1e-3)) / 1e9 if ms_fact > 0 else None
    out = {
        "metric": "p50 NMPC re-solve ms + IPM iters/s; Cholesky GB/s vs HBM roofline",
        "value": iters / elapsed,
        "unit": "IPM iters/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": elapsed * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "distillation 40 trays, horizon 100, dt 0.05, alpha~U(2,3), sinusoidal zF, "
                               "warm-started re-solves", "seed": a.seed, "n": p.n, "nnz_kkt": nk,
                   "nnz_l": sym["nnz_l"], "supernodes": sym["n_supernodes"], "etree_depth": sym["depth"]},
        "p50_resolve_ms": _percentile(lat, 50),
        "p99_resolve_ms": _percentile(lat, 99),
        "resolves_per_s": a.steps / elapsed,
        "iters_per_resolve": iters / a.steps,
        "first_solve_ms": t_first * 1e3,
        "analyze_ms": t_an * 1e3,
        "nonzero_status": sum(1 for s in statuses if s != 0),
        "phase_ms_per_resolve": {k: v / a.steps for k, v in phase.items()},
        "cholesky_gflops": gflops,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBPS) if achieved else None, "traffic": measured_traffic(),
                     "kernel": "numeric supernodal factorization (all levels of one factorization)",
                     "bytes_per_unit": bytes_per_factor},
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.seed, a.cpu_budget)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
