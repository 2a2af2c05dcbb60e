#!/usr/bin/env python3
"""NMPC re-solve benchmark on one MI355X.

Workload (default): distillation column, 40 trays (42 states) + reflux and
boilup, horizon 100 implicit-Euler stages of 0.05, alpha ~ U(2,3) from the
seed, sinusoidal feed-composition disturbance, warm-started receding-horizon
re-solves with one symbolic analysis.  A step is one warm re-solve: parameter
upload, every interior-point iteration on the GPU (eval, assembly, supernodal
Cholesky, solves, line search), and the download of u_1 and x_1 for the plant.
The first solve (analyze + cold start) is reported on its own.

Prints one JSON line.  --gpus N with N > 1 is refused: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBPS = 8000.0
FP64_PEAK_TFLOPS = 78.6


TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "factor_distill_medium_hbm_traffic.txt")
PLATE_TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                                  "factor_plate_32x32x50_hbm_traffic.txt")


def measured_traffic(path=TRAFFIC_FILE):
    """HBM bytes per factorization from a committed counter summary, or None
    when a source of the factorization kernels changed since the counters were
    taken (the summary lists the files and their SHA-256)."""
    import hashlib
    try:
        kv = {}
        for line in open(path):
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
        root = os.path.join(os.path.dirname(path), "..")
        files, shas = kv["source_file"].split(), kv["source_sha256"].split()
        if len(files) != len(shas):
            return None
        for f, h in zip(files, shas):
            if hashlib.sha256(open(os.path.join(root, f), "rb").read()).hexdigest() != h:
                return None
        return float(kv["bytes_per_factorization"])
    except (OSError, KeyError, ValueError):
        return None


def _progress(msg):
    """One line on stderr per finished stage (long runs report as they go)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _percentile(v, q):
    return float(np.percentile(np.asarray(v, dtype=float), q)) if len(v) else float("nan")


def cpu_baseline(seed: int, budget_s: float):
    """The oracle's interior-point method on the host, bounded sample of the
    same workload: one cold solve (untimed set-up), then warm re-solves until
    the time budget is spent."""
    from oracle.distillation import DistillationOCP
    from oracle.ipm import LiftedIPM
    from workloads import distillation_workload
    import contextlib
    # BLAS threads: the host's cores, bounded by the thread budget the
    # environment gives this process (OMP_NUM_THREADS), set with threadpoolctl
    want = max(1, min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))))
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        limiter = threadpool_limits(limits=want)
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        blas = sorted({f"{i.get('internal_api')} {i.get('version')}" for i in threadpool_info()})
    except Exception:
        limiter, threads, blas = contextlib.nullcontext(), 1, []
    with limiter:
        return _cpu_baseline(seed, budget_s, threads, blas)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _numpy_blas():
    """numpy's build configuration, BLAS/LAPACK entries only."""
    try:
        cfg = np.show_config(mode="dicts")
        deps = cfg.get("Build Dependencies", {})
        return {k: {kk: vv for kk, vv in v.items() if kk in ("name", "version", "found")}
                for k, v in deps.items() if k in ("blas", "lapack")}
    except Exception:
        return None


def _cpu_baseline(seed, budget_s, threads, blas):
    from oracle.distillation import DistillationOCP
    from oracle.ipm import LiftedIPM
    from workloads import distillation_workload
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
            "kind": "oracle", "cpu_model": _cpu_model(), "os_cpu_count": os.cpu_count(),
            "blas_threadpools": blas, "numpy_blas": _numpy_blas(),
            "sample": f"medium distillation seed {seed}: {len(times)} warm re-solves after one cold solve "
                      f"({iters} IPM iterations, {tot:.1f} s)",
            "p50_resolve_ms": _percentile([t * 1e3 for t in times], 50)}


def run_ablation(N, make, params, resolves, label):
    """The paper's structure-reuse ablation on one workload: the same closed
    loop of re-solves run four ways, symbolic analysis once (the method) or
    before every solve (a new handle analyzed each time, the warm start carried
    over with the iterate), and warm or cold starts.  Times are host wall time
    per re-solve, analysis and device set-up included where they run."""
    out = {"workload": label, "resolves": resolves}
    for every in (False, True):
        for warm in (True, False):
            p = make()
            p.analyze()
            params(p, -1, None, None)
            r = p.solve(warm=False)
            u1, x1 = p.first_stage()
            lat, an, iters, bad = [], [], 0, 0
            for k in range(resolves):
                t = time.perf_counter()
                if every:
                    it = p.get_iterate() if warm else None
                    p.close()
                    p = make()
                    ta = time.perf_counter()
                    p.analyze()
                    an.append((time.perf_counter() - ta) * 1e3)
                    params(p, k, u1, x1)
                    if warm:
                        p.set_iterate(it["y"], it["s"], it["omega"], it["beta"], it["zL"], it["zU"])
                else:
                    params(p, k, u1, x1)
                r = p.solve(warm=warm)
                u1, x1 = p.first_stage()
                lat.append((time.perf_counter() - t) * 1e3)
                iters += r.iters
                bad += r.status != 0
            p.close()
            key = ("analyze_every_solve" if every else "analyze_once") + ("_warm" if warm else "_cold")
            out[key] = {"p50_resolve_ms": _percentile(lat, 50), "mean_resolve_ms": float(np.mean(lat)),
                        "iters_per_resolve": iters / resolves, "nonzero_status": bad}
            if every:
                out[key]["mean_analyze_ms"] = float(np.mean(an))
    base = out["analyze_once_warm"]["mean_resolve_ms"]
    out["slowdown_vs_analyze_once_warm"] = {k: v["mean_resolve_ms"] / base for k, v in out.items()
                                            if isinstance(v, dict) and "mean_resolve_ms" in v}
    _progress(f"ablation: {label}")
    return out


def ablations(N):
    from workloads import distillation_workload, plate_workload

    def column(kind, resolves):
        w = distillation_workload(kind, 0, n_resolves=resolves + 1)
        sp = [w.xD_sp, w.xB_sp]

        def make():
            return N.Problem(N.distillation_structure(w.N, w.H, w.dt, w.alpha, F=w.F, rho=w.rho))

        def params(p, k, u1, x1):
            if k < 0:
                p.set_parameters(w.x0, setpoint=sp, traj=w.zF(0), u_prev=w.u_prev0)
            else:
                p.set_parameters(w.next_measurement(x1, k), setpoint=sp, traj=w.zF(k + 1), u_prev=u1)
        return make, params, f"distillation {w.N} trays, horizon {w.H}, seed 0"

    def plate(resolves):
        w = plate_workload("large", 0)

        def make():
            return N.Problem(N.plate_structure(w.G, w.H, w.dt, t_hi=w.T_hi, c_lo=w.u_lo, c_hi=w.u_hi))

        def params(p, k, u1, x1):
            if k < 0:
                p.set_parameters(w.T0, setpoint=w.target, u_prev=np.full(16, 0.5 * (w.u_lo + w.u_hi)))
            else:
                p.set_parameters(x1, setpoint=w.target, u_prev=u1)
        return make, params, f"heated plate {w.G}x{w.G}, horizon {w.H}, seed 0"

    out = {}
    for name, (mk, pr, lab), R in (("small", column("small", 5), 5), ("medium", column("medium", 10), 10),
                                     ("plate", plate(3), 3)):
        out[name] = run_ablation(N, mk, pr, R, lab)
    return out


def trisolve_rate(p, nnz_l, reps=20):
    """Forward and back substitution with the held factor through
    nmpc_linear_solve: host wall time per call (the right-hand side and the
    solution cross PCIe, 16 n bytes) and 16 nnz(L) bytes (L read once forward,
    once backward) over it."""
    rng = np.random.default_rng(0)
    b = rng.normal(size=p.n)
    p.linear_solve(b)
    t = time.perf_counter()
    for _ in range(reps):
        p.linear_solve(b)
    dt = (time.perf_counter() - t) / reps
    return {"ms_per_solve": dt * 1e3, "gbps": 16.0 * nnz_l / dt / 1e9, "bytes_per_solve": 16.0 * nnz_l,
            "note": "host wall time incl. the 16 n bytes of right-hand side and solution over PCIe"}


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Device-to-device copy of nbytes (read + write counted), HIP events."""
    import torch
    n = nbytes // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return {"bytes": 2 * n * 8, "ms": ms, "gbps": 2 * n * 8 / (ms * 1e-3) / 1e9}


PAPER_CASE_STUDY_TOTAL_S = 3.00   # Section 4.3: distillation, WS+PU, RTX 6000 Ada (context only)


def run_case_study(N, eager=False):
    """The paper's distillation case study (Section 4.1, Table 1): 32 trays,
    reflux-ratio control, horizon 90 stages of 2 s, closed loop of 150 NMPC
    steps from t = 0 to 300 s, plant = the model, symbolic analysis once and
    warm starts (the paper's WS+PU configuration).  Timed end to end: the
    analysis, the cold first solve and every step (parameter upload, solve,
    first-stage download)."""
    from workloads import reflux_workload
    w = reflux_workload()
    opts = N.default_options(graph=0 if eager else 1)
    t0 = time.perf_counter()
    p = N.Problem(N.reflux_structure(w.H, dt=w.dt))
    p.analyze()
    t_an = time.perf_counter() - t0
    x0, up = w.x0.copy(), np.array([w.u_prev0])
    lat, iters, bad = [], 0, 0
    for k in range(w.n_steps):
        t = time.perf_counter()
        p.set_parameters(x0, setpoint=[w.xbar, w.ubar], u_prev=up)
        r = p.solve(warm=k > 0, options=opts)
        u1, x1 = p.first_stage()
        lat.append((time.perf_counter() - t) * 1e3)
        iters += r.iters
        bad += r.status != 0
        x0, up = x1, u1
    total = time.perf_counter() - t0
    _progress(f"case study: {w.n_steps} NMPC steps in {total:.2f} s")
    return {"workload": f"distillation case study of Section 4.1 (Table 1): {w.N} trays, feed tray {w.Nf}, "
                        f"reflux-ratio control, horizon {w.H} x {w.dt} s, {w.n_steps} NMPC steps, plant = model",
            "n": p.n, "total_s": total, "analyze_ms": t_an * 1e3, "first_solve_ms": lat[0],
            "p50_step_ms": _percentile(lat[1:], 50), "p99_step_ms": _percentile(lat[1:], 99),
            "iters_total": iters, "nonzero_status": bad, "final_x1": float(x0[0]), "final_u": float(up[0]),
            "paper_total_s": PAPER_CASE_STUDY_TOTAL_S,
            "paper_hardware": "NVIDIA RTX 6000 Ada, MadNLP + cuDSS, WS+PU (context only)"}


def _loop_rate(N, p, w, steps, warmup, eager):
    """The headline re-solve loop on one problem: cold solve, warm-up, then
    `steps` timed warm re-solves (parameter upload, solve, first-stage
    download), each step measured from its own first stage."""
    import torch
    sp = [w.xD_sp, w.xB_sp]
    opts = N.default_options(timing=1, graph=0 if eager else 1)
    p.set_parameters(w.x0, setpoint=sp, traj=w.zF(0), u_prev=w.u_prev0)
    r0 = p.solve(warm=False)
    u1, x1 = p.first_stage()
    lat, iters, ms_eval, bad = [], 0, 0.0, int(r0.status != 0)
    torch.cuda.synchronize()
    t_begin = None
    for k in range(warmup + steps):
        if k == warmup:
            torch.cuda.synchronize()
            t_begin = time.perf_counter()
        t = time.perf_counter()
        p.set_parameters(w.next_measurement(x1, k), setpoint=sp, traj=w.zF(k + 1), u_prev=u1)
        r = p.solve(warm=True, options=opts)
        u1, x1 = p.first_stage()
        if k >= warmup:
            lat.append((time.perf_counter() - t) * 1e3)
            iters += r.iters
            ms_eval += r.ms_eval
            bad += r.status != 0
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_begin
    return {"iters_per_s": iters / elapsed, "p50_resolve_ms": _percentile(lat, 50),
            "p99_resolve_ms": _percentile(lat, 99), "iters": iters, "eval_ms_per_resolve": ms_eval / steps,
            "cold_iters": r0.iters, "nonzero_status": bad}


def _plate_summary(r):
    keys = ("p50_resolve_ms", "p99_resolve_ms", "iters_per_s", "iters_per_resolve", "nonzero_status",
            "cold_iters", "cold_status", "factor_ms", "phase_ms_per_resolve")
    return {k: r[k] for k in keys}


def run_front_end(N, steps=30, warmup=2, eager=False, plate_hand=None):
    """The headline workload written with the stage-pattern front end (its
    kernels generated from the stage expressions, as a stage model and as
    index-data patterns) beside the hand-written DISTILLATION family: the
    same closed re-solve loop on each; the workload
    plate written with index-data patterns beside the hand-written
    HEATED_PLATE family (plate_hand: that family's run_plate result when the
    caller has one); and the paper's case study (150 NMPC steps) through the
    generated case-study model and its index-data pattern form."""
    from paper_2606_04725_amd import simd, simd_models as SM
    from workloads import distillation_workload, reflux_workload
    w = distillation_workload("medium", 0, n_resolves=warmup + steps + 1)
    args = dict(F=w.F, rho=w.rho, x_lo=w.x_lo, x_hi=w.x_hi, u_lo=w.u_lo, u_hi=w.u_hi)
    g = simd.compile(SM.distillation_model(w.N, w.alpha, **args))
    gp = simd.compile(SM.distillation_pattern_model(w.N, w.alpha, **args))
    out = {"workload": f"distillation {w.N} trays, horizon {w.H}, dt {w.dt}, seed 0, {steps} warm re-solves "
                       f"(same loop as the headline line, without autotuning)"}
    for name, st in (("generated", N.stage_model_structure(g, w.H, w.dt)),
                     ("pattern", N.stage_model_structure(gp, w.H, w.dt)),
                     ("hand_written", N.distillation_structure(w.N, w.H, w.dt, w.alpha, F=w.F, rho=w.rho))):
        p = N.Problem(st)
        p.analyze()
        out[name] = _loop_rate(N, p, w, steps, warmup, eager)
        p.close()
    _progress(f"front end: generated {out['generated']['iters_per_s']:.0f} iters/s, pattern "
              f"{out['pattern']['iters_per_s']:.0f}, hand-written {out['hand_written']['iters_per_s']:.0f} iters/s")
    hand = plate_hand if plate_hand is not None else run_plate(N, eager=eager)
    out["plate"] = {"workload": hand["workload"] + "; generated = one stencil pattern and one tracking pattern",
                    "generated": _plate_summary(run_plate(N, eager=eager, model="pattern")),
                    "hand_written": _plate_summary(hand)}
    _progress(f"front end plate: generated p50 {out['plate']['generated']['p50_resolve_ms']:.2f} ms, "
              f"hand-written p50 {out['plate']['hand_written']['p50_resolve_ms']:.2f} ms")
    rw = reflux_workload()
    opts = N.default_options(graph=0 if eager else 1)
    for key, make in (("case_study_generated", SM.reflux_model), ("case_study_pattern", SM.reflux_pattern_model)):
        gr = simd.compile(make(N=rw.N, Nf=rw.Nf, D=rw.D, F=rw.F, alpha=rw.alpha, xf=rw.xf, Ac=rw.Ac, At=rw.At,
                               Ar=rw.Ar, w_u=rw.w_u))
        t0 = time.perf_counter()
        p = N.Problem(N.stage_model_structure(gr, rw.H, rw.dt))
        p.analyze()
        x0, up = rw.x0.copy(), np.array([rw.u_prev0])
        iters, bad = 0, 0
        for k in range(rw.n_steps):
            p.set_parameters(x0, setpoint=[rw.xbar, rw.ubar], u_prev=up)
            r = p.solve(warm=k > 0, options=opts)
            up, x0 = p.first_stage()
            iters += r.iters
            bad += r.status != 0
        out[key] = {"total_s": time.perf_counter() - t0, "iters_total": iters, "nonzero_status": bad,
                    "final_x1": float(x0[0]), "final_u": float(up[0])}
        p.close()
    return out


def run_device_loop(N, steps=50, warmup=2, passes=(1, 2, 3)):
    """Algorithm 1's loop with plant = model and the workload's measurement
    noise, driven from the host (set_parameters, solve, first_stage per step)
    and on the device (nmpc_closed_loop_dev: the parameter update and the
    first passes of each re-solve in one captured graph), on the headline
    column (40 trays, horizon 100) and the case study of Section 4.1."""
    import torch
    from workloads import distillation_workload, reflux_workload
    w = distillation_workload("medium", 0, n_resolves=warmup + steps + 1)
    sp = [w.xD_sp, w.xB_sp]
    dev = torch.device("cuda")
    traj = torch.tensor(np.array([w.zF(k + 1) for k in range(warmup + steps)]), dtype=torch.float64, device=dev)
    noise = torch.tensor(w.resolve_noise[:warmup + steps], dtype=torch.float64, device=dev)

    def fresh():
        p = N.Problem(N.distillation_structure(w.N, w.H, w.dt, w.alpha, F=w.F, rho=w.rho))
        p.analyze()
        p.autotune(reps=3)
        p.set_parameters(w.x0, setpoint=sp, traj=w.zF(0), u_prev=w.u_prev0)
        assert p.solve(warm=False).status == 0
        return p

    out = {"workload": f"distillation {w.N} trays, horizon {w.H}, seed 0: {steps} warm re-solves after {warmup}, "
                       f"measurement = predicted x1 + the workload's noise"}
    p = fresh()
    u1, x1 = p.first_stage()
    iters = 0
    for k in range(warmup + steps):
        if k == warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        p.set_parameters(w.next_measurement(x1, k), setpoint=sp, traj=w.zF(k + 1), u_prev=u1)
        r = p.solve(warm=True)
        u1, x1 = p.first_stage()
        if k >= warmup:
            iters += r.iters
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["host_loop"] = {"iters_per_s": iters / el, "ms_per_resolve": el * 1e3 / steps, "iters": iters}
    p.close()
    for ppg in passes:
        p = fresh()
        rc, _, _ = p.closed_loop_dev(warmup, traj.data_ptr(), noise.data_ptr(), passes_per_step=ppg)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, done, it = p.closed_loop_dev(steps, traj[warmup:].data_ptr(), noise[warmup:].data_ptr(),
                                         passes_per_step=ppg)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[f"device_loop_{ppg}_passes"] = {"iters_per_s": it / el, "ms_per_resolve": el * 1e3 / steps,
                                            "iters": it, "status": rc, "steps": done}
        p.close()
    # the case study, device loop (analysis and the cold first solve included)
    rw = reflux_workload()
    t0 = time.perf_counter()
    p = N.Problem(N.reflux_structure(rw.H, dt=rw.dt))
    p.analyze()
    p.set_parameters(rw.x0, setpoint=[rw.xbar, rw.ubar], u_prev=[rw.u_prev0])
    r0 = p.solve(warm=False)
    rc, done, it = p.closed_loop_dev(rw.n_steps - 1, passes_per_step=2)
    torch.cuda.synchronize()
    out["case_study_device_loop"] = {"total_s": time.perf_counter() - t0, "iters_total": r0.iters + it,
                                     "status": rc, "steps": done + 1}
    p.close()
    _progress(f"device loop: host {out['host_loop']['iters_per_s']:.0f} iters/s, device (2 passes) "
              f"{out['device_loop_2_passes']['iters_per_s']:.0f} iters/s")
    return out


PAPER_PLATE_CASE_TOTAL_S = 3.28   # Table 3: InfiniteExaModels + MadNLP + cuDSS, WS + PU, PDE plate


def run_plate_case_study(N, eager=False, model="stage"):
    """The heated-plate case study of Section 4.2 (Table 2) written with the
    stage-pattern front end: 21 x 21 grid, horizon 12 stages of 0.08 s, 38
    NMPC steps from t = 0 to 3 s with the setpoint schedule 58 / 55 / 63, plant
    = model, symbolic analysis once and warm starts.  Timed end to end like
    the distillation case study.  model: "stage" (one generated case per grid
    point) or "pattern" (index-data patterns); the pattern form's run is
    reported under "pattern_model"."""
    from paper_2606_04725_amd import simd, simd_models as SM
    from workloads import plate_case_workload
    w = plate_case_workload()
    make = SM.plate_case_model if model == "stage" else SM.plate_case_pattern_model
    g = simd.compile(make(n=w.n, alpha=w.alpha, Tb=w.Tb, loss=w.loss, rho=w.rho, Q_lo=w.Q_lo, q_scale=w.q_scale,
                          dt=w.dt))
    opts = N.default_options(graph=0 if eager else 1)
    t0 = time.perf_counter()
    p = N.Problem(N.stage_model_structure(g, w.H, w.dt))
    p.analyze()
    t_an = time.perf_counter() - t0
    nx = p.nx
    x0, up = np.full(nx, w.T0), np.array([w.Q_prev0 / w.q_scale])
    lat, iters, bad, qs, means = [], 0, 0, [], []
    region = None
    for k in range(w.n_steps):
        t = time.perf_counter()
        p.set_parameters(x0, traj=w.traj(k), u_prev=up)
        r = p.solve(warm=k > 0, options=opts)
        u1, x1 = p.first_stage()
        lat.append((time.perf_counter() - t) * 1e3)
        iters += r.iters
        bad += r.status != 0
        x0, up = x1, u1
        qs.append(float(u1[0]) * w.q_scale)
        if region is None:
            gpts = w.n - 2
            xs = -1.0 + (2.0 / (w.n - 1)) * np.arange(1, w.n - 1)
            inside = np.abs(xs) <= 0.5 + 1e-12
            region = np.outer(inside, inside).reshape(-1)
        means.append(float(np.mean(x1[region])))
    total = time.perf_counter() - t0
    _progress(f"plate case study ({model} model): {w.n_steps} NMPC steps in {total:.2f} s")
    if model != "stage":
        return {"total_s": total, "p50_step_ms": _percentile(lat[1:], 50), "iters_total": iters,
                "nonzero_status": bad, "Q_first_last": [qs[0], qs[-1]]}
    out = {"workload": f"heated-plate case study of Section 4.2 (Table 2): {w.n} x {w.n} grid, horizon {w.H} x "
                        f"{w.dt} s, {w.n_steps} NMPC steps, setpoint 58 / 55 / 63, plant = model, loss term read "
                        f"as {w.loss}", "n": p.n, "total_s": total, "analyze_ms": t_an * 1e3,
            "first_solve_ms": lat[0], "p50_step_ms": _percentile(lat[1:], 50),
            "p99_step_ms": _percentile(lat[1:], 99), "iters_total": iters, "nonzero_status": bad,
            "Q_first_last": [qs[0], qs[-1]], "region_mean_at_steps_6_18_37": [means[6], means[18], means[-1]],
            "paper_total_s": PAPER_PLATE_CASE_TOTAL_S,
            "paper_hardware": "NVIDIA RTX 6000 Ada, MadNLP + cuDSS, WS+PU (context only)"}
    out["pattern_model"] = run_plate_case_study(N, eager=eager, model="pattern")
    return out


def run_mismatch(N, steps=30, seed=0, factor=1.08, eager=False):
    """Closed loop of the small column against a plant whose relative
    volatility is the model's times ``factor`` (plant-model mismatch), beside
    the same loop with a matched plant: warm re-solves per step, measured
    (not predicted) next state, tracking offsets at the end."""
    from paper_2606_04725_amd.plant import DistillationPlant
    from workloads import distillation_workload
    w = distillation_workload("small", seed)
    opts = N.default_options(graph=0 if eager else 1)
    out = {"workload": f"distillation 10 trays, horizon 20, {steps} closed-loop steps, plant alpha = model alpha "
                       f"x {factor} vs matched"}
    for name, alpha in (("matched", w.alpha), ("mismatched", factor * w.alpha)):
        plant = DistillationPlant(w.N, alpha, w.dt, F=w.F)
        p = N.Problem(N.distillation_structure(w.N, w.H, w.dt, w.alpha, F=w.F, rho=w.rho))
        p.analyze()
        x, up = w.x0.copy(), w.u_prev0.copy()
        lat, iters, bad = [], 0, 0
        for k in range(steps):
            t = time.perf_counter()
            p.set_parameters(x, setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(k), u_prev=up)
            r = p.solve(warm=k > 0, options=opts)
            u1, _ = p.first_stage()
            lat.append((time.perf_counter() - t) * 1e3)
            iters += r.iters
            bad += r.status != 0
            x = plant.step(x, u1, zF=float(w.zF(k)[0]))
            up = u1
        out[name] = {"p50_resolve_ms": _percentile(lat[1:], 50), "iters_per_resolve": iters / steps,
                     "nonzero_status": bad, "final_top_offset": float(x[0] - w.xD_sp),
                     "final_bottom_offset": float(x[-1] - w.xB_sp)}
    _progress("plant-model mismatch loop")
    return out


def run_batched(N, count=64, base_seed=1000, rounds=10, eager=False):
    """Batched form: 64 ragged distillation instances (trays U{20..60}, horizons
    U{40..120}, alpha U(2,3), own setpoints and noise), one cold solve, then
    `rounds` warm re-solve rounds; the same instances solved one by one on
    separate handles are timed beside it.  Per-instance latency of a batched
    re-solve is the wall time of the round it belongs to."""
    from workloads import batch_distillation_workloads
    ws = batch_distillation_workloads(count, base_seed)
    opts = N.default_options(graph=0 if eager else 1)

    def make():
        ps = []
        for w in ws:
            q = N.Problem(N.distillation_structure(w.N, w.H, w.dt, w.alpha, F=w.F, rho=w.rho))
            q.analyze()
            q.autotune(reps=2)
            q.set_parameters(w.x0, setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(0), u_prev=w.u_prev0)
            ps.append(q)
        return ps

    def params(q, w, u1, x1, k):
        q.set_parameters(w.next_measurement(x1, k), setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(k + 1), u_prev=u1)

    t0 = time.perf_counter()
    pb = make()
    t_an = time.perf_counter() - t0
    _progress(f"batch: {count} problems analyzed and tuned")
    b = N.Batch(pb)
    t0 = time.perf_counter()
    rc, res0 = b.solve(warm=False, options=opts)
    t_cold = time.perf_counter() - t0
    cold_bad = [i for i, r in enumerate(res0) if r.status != 0]
    _progress(f"batch: cold solve done, {len(cold_bad)} nonzero status")
    fs = [q.first_stage() for q in pb]
    lat_b, it_b, st_b = [], 0, []
    t_begin = time.perf_counter()
    for k in range(rounds):
        t = time.perf_counter()
        for q, w, (u1, x1) in zip(pb, ws, fs):
            params(q, w, u1, x1, k)
        rc, res = b.solve(warm=True, options=opts)
        fs = [q.first_stage() for q in pb]
        dt = time.perf_counter() - t
        lat_b += [dt * 1e3] * count
        it_b += sum(r.iters for r in res)
        st_b += [r.status for r in res]
    el_b = time.perf_counter() - t_begin
    b.close()
    _progress("batch: batched re-solves done")
    ps = make()
    for q in ps:
        q.solve(warm=False, options=opts)
    fs = [q.first_stage() for q in ps]
    lat_s, it_s, st_s = [], 0, []
    t_begin = time.perf_counter()
    for k in range(rounds):
        for i, (q, w) in enumerate(zip(ps, ws)):
            t = time.perf_counter()
            params(q, w, fs[i][0], fs[i][1], k)
            r = q.solve(warm=True, options=opts)
            fs[i] = q.first_stage()
            lat_s.append((time.perf_counter() - t) * 1e3)
            it_s += r.iters
            st_s.append(r.status)
    el_s = time.perf_counter() - t_begin
    _progress("batch: one-by-one re-solves done")
    n_tot = sum(q.n for q in pb)
    return {"workload": f"{count} distillation instances, trays U{{20..60}}, horizons U{{40..120}}, alpha U(2,3), "
                        f"seeds {base_seed}..{base_seed + count - 1}, {rounds} warm re-solve rounds",
            "n_total": n_tot, "analyze_s": t_an, "cold_batch_ms": t_cold * 1e3,
            "cold_iters_max": max(r.iters for r in res0), "cold_nonzero_status": cold_bad,
            "resolves_per_s": count * rounds / el_b, "iters_per_s": it_b / el_b,
            "p50_instance_ms": _percentile(lat_b, 50), "p99_instance_ms": _percentile(lat_b, 99),
            "nonzero_status": sum(1 for s_ in st_b if s_ != 0),
            "sequential": {"resolves_per_s": count * rounds / el_s, "iters_per_s": it_s / el_s,
                           "p50_instance_ms": _percentile(lat_s, 50), "p99_instance_ms": _percentile(lat_s, 99),
                           "nonzero_status": sum(1 for s_ in st_s if s_ != 0)},
            "speedup_vs_sequential": el_s / el_b}


def run_small(N, seeds=20, resolves=5, eager=False):
    """Small column (10 trays, horizon 20, dt 0.1): per seed one analyze + cold
    solve (reported apart), then warm re-solves with the plant stepped by the
    model plus measurement noise; p50 / p99 over the warm re-solves."""
    from workloads import distillation_workload
    opts = N.default_options(graph=0 if eager else 1)
    lat, first, iters, statuses = [], [], 0, []
    t_all = 0.0
    for seed in range(seeds):
        w = distillation_workload("small", seed, n_resolves=resolves + 1)
        t0 = time.perf_counter()
        p = N.Problem(N.distillation_structure(w.N, w.H, w.dt, w.alpha, F=w.F, rho=w.rho))
        p.analyze()
        sp = [w.xD_sp, w.xB_sp]
        p.set_parameters(w.x0, setpoint=sp, traj=w.zF(0), u_prev=w.u_prev0)
        r0 = p.solve(warm=False, options=opts)
        u1, x1 = p.first_stage()
        first.append((time.perf_counter() - t0) * 1e3)
        statuses.append(r0.status)
        for k in range(resolves):
            t = time.perf_counter()
            p.set_parameters(w.next_measurement(x1, k), setpoint=sp, traj=w.zF(k + 1), u_prev=u1)
            r = p.solve(warm=True, options=opts)
            u1, x1 = p.first_stage()
            dt = time.perf_counter() - t
            lat.append(dt * 1e3)
            t_all += dt
            iters += r.iters
            statuses.append(r.status)
        p.close()
    _progress(f"small column: {seeds} seeds x {resolves} warm re-solves")
    return {"workload": f"distillation 10 trays, horizon 20, dt 0.1, seeds 0..{seeds - 1}, {resolves} warm re-solves each",
            "p50_resolve_ms": _percentile(lat, 50), "p99_resolve_ms": _percentile(lat, 99),
            "iters_per_s": iters / t_all, "iters_per_resolve": iters / len(lat),
            "p50_first_solve_ms": _percentile(first, 50), "nonzero_status": sum(1 for s_ in statuses if s_ != 0)}


def run_plate(N, G=32, H=50, seed=0, resolves=20, adjoint=False, eager=False, model="hand_written"):
    """Heated plate: G x G grid, horizon H, dt 0.01, 16 heaters in [0, 1],
    T <= 1.5, Gaussian-bump target from the seed, T0 = 0.  One analyze and cold
    solve, then warm re-solves where the plant is the model (the next
    measurement is the predicted first-stage field).  With adjoint, after each
    re-solve d u1*/d x0 (nu x G^2) and d f*/d setpoint (G^2) are computed.
    model: the hand-written HEATED_PLATE family, or "pattern" for the same
    plate written with the front end's index-data patterns."""
    from workloads import plate_workload
    w = plate_workload("large", seed, G=G, H=H)
    if model == "pattern":
        from paper_2606_04725_amd import simd, simd_models as SM
        st = N.stage_model_structure(simd.compile(SM.plate_pattern_model(G)), H, w.dt)
    else:
        st = N.plate_structure(G, H, w.dt, t_hi=w.T_hi, c_lo=w.u_lo, c_hi=w.u_hi)
    p = N.Problem(st)
    t0 = time.perf_counter()
    p.analyze()
    t_an = time.perf_counter() - t0
    sym = p.symbolic_sizes()
    p.set_parameters(w.T0, setpoint=w.target, u_prev=np.full(16, 0.5 * (w.u_lo + w.u_hi)))
    opts = N.default_options(timing=1, graph=0 if eager else 1)
    t0 = time.perf_counter()
    r0 = p.solve(warm=False, options=opts)
    t_cold = time.perf_counter() - t0
    _progress(f"plate {G}x{G}x{H}: cold solve status {r0.status}, {r0.iters} iterations")
    u1, x1 = p.first_stage()
    lat, lat_adj, lat_adj2, lat_vjp, iters, facts, ms_fact, statuses = [], [], [], [], 0, 0, 0.0, []
    phase = dict(eval=0.0, assemble=0.0, factor=0.0, solve=0.0, linesearch=0.0)
    if adjoint:
        import torch
        from paper_2606_04725_amd.autograd import NMPCSolve
        cuda = torch.device("cuda:0")
        sp_t = torch.tensor(w.target, dtype=torch.float64, device=cuda, requires_grad=True)
    for k in range(resolves):
        if adjoint:
            # the differentiated form: forward through the autograd function on
            # device tensors, d f*/d setpoint by its backward (one adjoint
            # solve), d u1*/d x0 by the 16-seed Jacobian of the same solution
            x0_t = torch.tensor(x1, dtype=torch.float64, device=cuda, requires_grad=True)
            up_t = torch.tensor(u1, dtype=torch.float64, device=cuda)
            t = time.perf_counter()
            u1_t, f_t = NMPCSolve.apply(p, x0_t, sp_t, None, up_t, True, opts)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t) * 1e3)
            r = p.last_result
            u1, x1 = p.first_stage()
            t = time.perf_counter()
            rc, J = p.jacobian_u1_x0()              # factors K at the solution, then 16 seeds
            lat_adj.append((time.perf_counter() - t) * 1e3)
            t = time.perf_counter()
            rc, J2 = p.jacobian_u1_x0()             # the kept factor: solves only
            lat_adj2.append((time.perf_counter() - t) * 1e3)
            t = time.perf_counter()
            (g_sp,) = torch.autograd.grad(f_t, sp_t)
            torch.cuda.synchronize()
            lat_vjp.append((time.perf_counter() - t) * 1e3)
        else:
            t = time.perf_counter()
            p.set_parameters(x1, u_prev=u1)
            r = p.solve(warm=True, options=opts)
            u1, x1 = p.first_stage()
            lat.append((time.perf_counter() - t) * 1e3)
        iters += r.iters
        facts += r.factorizations
        ms_fact += r.ms_factor
        statuses.append(r.status)
        for key in phase:
            phase[key] += getattr(r, "ms_" + key)
        _progress(f"plate {G}x{G}x{H}: re-solve {k + 1}/{resolves} status {r.status}")
    tot = sum(lat) / 1e3
    flops = float(sym["flops"])
    achieved = (facts * flops / (ms_fact * 1e-3)) / 1e12 if ms_fact > 0 else None
    out = {"workload": f"heated plate {G}x{G}, horizon {H}, dt {w.dt}, 16 heaters, seed {seed}, "
                       f"{resolves} warm re-solves (plant = model)",
           "n": p.n, "nnz_l": sym["nnz_l"], "supernodes": sym["n_supernodes"], "analyze_ms": t_an * 1e3,
           "cold_solve_ms": t_cold * 1e3, "cold_iters": r0.iters, "cold_status": r0.status,
           "p50_resolve_ms": _percentile(lat, 50), "p99_resolve_ms": _percentile(lat, 99),
           "iters_per_s": iters / tot if tot > 0 else None, "iters_per_resolve": iters / max(1, resolves),
           "nonzero_status": sum(1 for s_ in statuses if s_ != 0),
           "factor_ms": ms_fact / facts if facts else None,
           "phase_ms_per_resolve": {k_: v / max(1, resolves) for k_, v in phase.items()},
           "roofline": {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": (achieved / FP64_PEAK_TFLOPS) if achieved else None,
                        "traffic": (measured_traffic(PLATE_TRAFFIC_FILE)
                                    if (G, H, model, seed) == (32, 50, "hand_written", 0) and not adjoint else None),
                        "kernel": "numeric supernodal factorization (all launches of one factorization)",
                        "flops_per_unit": flops}}
    if adjoint:
        nnz_j = p.pattern_counts()[0]
        adj_bytes = 2 * 8.0 * sym["nnz_l"] + 8.0 * 16 * (p.n + nnz_j)
        solves_ms = _percentile(lat_adj2, 50)
        out["adjoint"] = {"p50_jacobian_u1_x0_ms": _percentile(lat_adj, 50),
                          "p50_jacobian_u1_x0_kept_factor_ms": solves_ms,
                          "p50_objective_setpoint_gradient_ms": _percentile(lat_vjp, 50),
                          "jacobian_shape": [16, G * G],
                          "jacobian_gbps": adj_bytes / (solves_ms * 1e-3) / 1e9,
                          "jacobian_bytes": adj_bytes,
                          "note": "forward through NMPCSolve on device tensors; d f/d setpoint by its backward; "
                                  "the first Jacobian call after a solve factors K at the solution (the "
                                  "interior-point method's last factor is one iterate earlier), the second "
                                  "reuses that factor; GB/s = (2*8*nnz L + 8*16*(n + nnz J)) / kept-factor time"}
    else:
        out["trisolve"] = trisolve_rate(p, sym["nnz_l"])
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--eager", action="store_true", help="launch every kernel from the host (no graph replay)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-instance batched form")
    ap.add_argument("--no-small", action="store_true", help="skip the small-column leg (10 trays, horizon 20)")
    ap.add_argument("--batch-only", action="store_true", help="only run the 64-instance batched form")
    ap.add_argument("--no-plate", action="store_true", help="skip the heated-plate workloads")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the analyze-once/every-solve and warm/cold ablation")
    ap.add_argument("--ablation-only", action="store_true", help="only run the ablation")
    ap.add_argument("--case-study-only", action="store_true",
                    help="only run the paper's two case studies (distillation 150 steps, heated plate 38 steps)")
    ap.add_argument("--plate-only", action="store_true", help="only run the heated-plate workloads")
    ap.add_argument("--plate-model", choices=("hand_written", "pattern"), default="hand_written",
                    help="with --plate-only: the hand-written plate family or the index-data pattern model")
    ap.add_argument("--device-loop-only", action="store_true",
                    help="only run the closed loop driven from the host vs on the device")
    ap.add_argument("--front-end-only", action="store_true",
                    help="only run the stage-pattern front end's legs (generated vs hand-written kernels)")
    ap.add_argument("--plate-case", choices=("plain", "adjoint", "both"), default="both",
                    help="with --plate-only: the 32x32x50 plate, the differentiated plate, or both")
    ap.add_argument("--adjoint-grid", type=int, default=64, help="grid of the differentiated form (64 in the full run)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline re-solve loop (its JSON line without the other legs)")
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
        print("bench.py: measures one GPU; runs on several GPUs are not supported", file=sys.stderr)
        return 2

    import torch
    from paper_2606_04725_amd import nmpc as N
    from workloads import distillation_workload

    if not torch.cuda.is_available() or not N.device_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    if a.case_study_only:
        print(json.dumps({"case_study": run_case_study(N, eager=a.eager),
                          "plate_case_study": run_plate_case_study(N, eager=a.eager)}), flush=True)
        return 0
    if a.ablation_only:
        print(json.dumps({"ablation": ablations(N)}), flush=True)
        return 0
    if a.device_loop_only:
        print(json.dumps({"device_loop": run_device_loop(N)}), flush=True)
        return 0
    if a.front_end_only:
        print(json.dumps({"front_end": run_front_end(N, eager=a.eager)}), flush=True)
        return 0
    if a.batch_only:
        print(json.dumps({"batched": run_batched(N, eager=a.eager)}), flush=True)
        return 0
    if a.plate_only:
        out = {}
        if a.plate_case in ("plain", "both"):
            out["plate"] = run_plate(N, eager=a.eager, model=a.plate_model)
        if a.plate_case in ("adjoint", "both"):
            out["plate_adjoint"] = run_plate(N, G=a.adjoint_grid, H=100, resolves=10, adjoint=True, eager=a.eager,
                                             model=a.plate_model)
        print(json.dumps(out), flush=True)
        return 0
    w = distillation_workload("medium", a.seed, n_resolves=a.warmup + a.steps + 1)
    p = N.Problem(N.distillation_structure(w.N, w.H, w.dt, w.alpha, F=w.F, rho=w.rho))
    sp = [w.xD_sp, w.xB_sp]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.analyze()
    t_an = time.perf_counter() - t0
    tuned = p.autotune(reps=3)
    p.set_parameters(w.x0, setpoint=sp, traj=w.zF(0), u_prev=w.u_prev0)
    r0 = p.solve(warm=False)
    u1, x1 = p.first_stage()
    sol = {"u1": u1, "x1": x1}
    t_first = time.perf_counter() - t0
    if r0.status != 0:
        print(f"bench.py: cold solve failed with status {r0.status}", file=sys.stderr)
        return 1
    _progress(f"distillation: analyze + cold solve {t_first:.2f} s, {r0.iters} iterations")
    sym = p.symbolic_sizes()
    opts = N.default_options(timing=1, graph=0 if a.eager else 1)

    def resolve(k):
        nonlocal sol
        x0 = w.next_measurement(sol["x1"], k)
        t = time.perf_counter()
        p.set_parameters(x0, setpoint=sp, traj=w.zF(k + 1), u_prev=sol["u1"])
        res = p.solve(warm=True, options=opts)
        u1, x1 = p.first_stage()
        sol = {"u1": u1, "x1": x1}
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
    _progress(f"distillation: {a.steps} timed re-solves in {elapsed:.2f} s")
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
        "autotuned_launches": tuned,
        "nonzero_status": sum(1 for s in statuses if s != 0),
        "phase_ms_per_resolve": {k: v / a.steps for k, v in phase.items()},
        "cholesky_gflops": gflops,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBPS) if achieved else None, "traffic": measured_traffic(),
                     "kernel": "numeric supernodal factorization (all levels of one factorization)",
                     "bytes_per_unit": bytes_per_factor},
    }
    if a.headline_only:
        print(json.dumps(out), flush=True)
        return 0
    out["trisolve"] = trisolve_rate(p, sym["nnz_l"])
    out["measured_copy"] = copy_bandwidth()
    if not a.no_small:
        out["small"] = run_small(N, eager=a.eager)
    if not a.no_batch:
        out["batched"] = run_batched(N, eager=a.eager)
    if not a.no_plate:
        out["plate"] = run_plate(N, eager=a.eager)
        out["plate_adjoint"] = run_plate(N, G=a.adjoint_grid, H=100, resolves=10, adjoint=True, eager=a.eager)
    out["case_study"] = run_case_study(N, eager=a.eager)
    out["plate_case_study"] = run_plate_case_study(N, eager=a.eager)
    out["mismatch"] = run_mismatch(N, eager=a.eager)
    out["front_end"] = run_front_end(N, eager=a.eager, plate_hand=out.get("plate"))
    out["device_loop"] = run_device_loop(N)
    if not a.no_ablation:
        out["ablation"] = ablations(N)
    if not a.no_cpu_baseline:
        _progress("cpu baseline (oracle) starts")
        out["cpu_baseline"] = cpu_baseline(a.seed, a.cpu_budget)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
