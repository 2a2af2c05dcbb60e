"""Batched form on the GPU, through the C ABI.

A batch runs every kernel over all of its instances at once and takes the
method's decisions per instance on the device; an instance's arithmetic is the
same as in its own solve (same kernels, same per-instance reduction order), so
batched and one-by-one results must be identical.  The graph-replayed pass
must match the eagerly launched pass exactly, and batched solutions must match
the oracle like single solves do.
"""
import sys

import numpy as np
import pytest

from paper_2606_04725_amd import nmpc as N
from oracle.distillation import DistillationOCP
from oracle.ipm import LiftedIPM
from oracle.kkt import kkt_error
from workloads import batch_distillation_workloads, distillation_workload

pytestmark = pytest.mark.gpu

RAGGED = [(4, 6), (10, 20), (17, 9), (25, 33), (8, 50), (2, 1)]


def _note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _problem(w):
    p = N.Problem(N.distillation_structure(w.N, w.H, w.dt, w.alpha, F=w.F, rho=w.rho))
    p.analyze()
    p.set_parameters(w.x0, setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(0), u_prev=w.u_prev0)
    return p


def _ragged_workloads():
    return [distillation_workload("small", 10 + i, N=n, H=h, n_resolves=3) for i, (n, h) in enumerate(RAGGED)]


def _next(p, w, k):
    u1, x1 = p.first_stage()
    p.set_parameters(w.next_measurement(x1, k), setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(k + 1), u_prev=u1)


def test_batch_matches_one_by_one():
    ws = _ragged_workloads()
    _note(f"batch vs one-by-one, sizes {RAGGED}")
    batched = [_problem(w) for w in ws]
    single = [_problem(w) for w in ws]
    b = N.Batch(batched)
    for k in range(3):
        rc, res = b.solve(warm=k > 0)
        assert rc == 0, [r.status for r in res]
        for i, (pb, ps) in enumerate(zip(batched, single)):
            r1 = ps.solve(warm=k > 0)
            assert r1.status == 0
            assert res[i].iters == r1.iters and res[i].factorizations == r1.factorizations, (k, i)
            assert res[i].ls_trials == r1.ls_trials
            sb, ss = pb.solution(), ps.solution()
            for key in ("y", "lam", "omega_d", "zL", "zU"):
                assert np.array_equal(sb[key], ss[key]), (k, i, key)
        for i, w in enumerate(ws):
            _next(batched[i], w, k)
            _next(single[i], w, k)
    b.close()


def test_graph_pass_matches_eager_pass():
    w = distillation_workload("small", 4, n_resolves=3)
    _note("graph vs eager, distillation 10 trays horizon 20")
    pg, pe = _problem(w), _problem(w)
    og, oe = N.default_options(graph=1), N.default_options(graph=0, timing=1)
    for k in range(3):
        rg = pg.solve(warm=k > 0, options=og)
        re = pe.solve(warm=k > 0, options=oe)
        assert rg.status == 0 and re.status == 0
        assert rg.iters == re.iters and rg.passes == re.passes
        sg, se = pg.solution(), pe.solution()
        assert np.array_equal(sg["y"], se["y"]) and np.array_equal(sg["lam"], se["lam"])
        assert re.ms_factor > 0.0
        _next(pg, w, k)
        _next(pe, w, k)


def test_graph_pass_with_timing_events():
    w = distillation_workload("small", 5)
    _note("graph with timing events")
    p = _problem(w)
    r = p.solve(warm=False, options=N.default_options(graph=1, timing=1))
    _note(f"timing_lost={r.timing_lost} passes={r.passes} ms_factor={r.ms_factor}")
    assert r.status == 0
    assert r.ms_factor > 0.0 and r.ms_eval > 0.0 and r.ms_solve > 0.0


@pytest.mark.parametrize("idx", [1, 3])
def test_batched_instances_match_oracle(idx):
    ws = _ragged_workloads()
    _note(f"batched instance {idx} vs oracle")
    ps = [_problem(w) for w in ws]
    b = N.Batch(ps)
    rc, res = b.solve(warm=False)
    assert rc == 0
    w = ws[idx]
    m = DistillationOCP.from_workload(w)
    m.set_parameters(x0=w.x0, zF=w.zF(0), u_prev=w.u_prev0)
    ipm = LiftedIPM(m)
    ref = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
    assert ref.status == 0
    sol = ps[idx].solution()
    assert res[idx].iters == ref.iters
    yr = ref.state.y
    assert np.max(np.abs(sol["y"] - yr)) / max(1.0, np.max(np.abs(yr))) <= 1e-6
    lam_ref = ref.state.omega[:m.m_c] - ref.state.omega[m.m_c:2 * m.m_c]
    assert np.max(np.abs(sol["lam"] - lam_ref)) / max(1.0, np.max(np.abs(lam_ref))) <= 1e-6
    b.close()


def test_full_batch_sampled():
    """The 64-instance ragged batch the benchmark times (trays U{20..60},
    horizons U{40..120}): every instance converges, sampled instances are
    identical to their one-by-one solves, and the oracle's evaluator certifies
    the original problem's optimality error at every instance."""
    ws = batch_distillation_workloads(64, 1000)
    _note("full 64-instance batch, cold + 1 warm")
    ps = [_problem(w) for w in ws]
    b = N.Batch(ps)
    rc, res = b.solve(warm=False)
    assert rc == 0, [r.status for r in res]
    sample = [0, 17, 63]
    for i in sample:
        q = _problem(ws[i])
        r1 = q.solve(warm=False)
        assert r1.iters == res[i].iters
        assert np.array_equal(q.solution()["y"], ps[i].solution()["y"])
    for i, (p, w) in enumerate(zip(ps, ws)):
        m = DistillationOCP.from_workload(w)
        m.set_parameters(x0=w.x0, zF=w.zF(0), u_prev=w.u_prev0)
        s = p.solution()
        E = kkt_error(m, s["y"], s["lam"], s["omega_d"], s["zL"], s["zU"])
        assert E["max"] <= 1e-8, (i, E)
    for i, w in enumerate(ws):
        _next(ps[i], w, 0)
    rc, res = b.solve(warm=True)
    assert rc == 0, [r.status for r in res]
    assert max(r.iters for r in res) < 100
    b.close()


def test_autotuned_solve_keeps_parity():
    """The autotuner only picks among variants of the front kernel: the solve
    after tuning still matches the oracle, and a second problem of the same
    structure takes the cached choice."""
    w = distillation_workload("small", 13, N=25, H=33, n_resolves=1)
    _note("autotune N=25 H=33")
    p = _problem(w)
    p.autotune(reps=2)
    r = p.solve(warm=False)
    assert r.status == 0
    m = DistillationOCP.from_workload(w)
    m.set_parameters(x0=w.x0, zF=w.zF(0), u_prev=w.u_prev0)
    ipm = LiftedIPM(m)
    ref = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
    assert ref.status == 0 and r.iters == ref.iters
    sol = p.solution()
    yr = ref.state.y
    assert np.max(np.abs(sol["y"] - yr)) / max(1.0, np.max(np.abs(yr))) <= 1e-6
    lam_ref = ref.state.omega[:m.m_c] - ref.state.omega[m.m_c:2 * m.m_c]
    assert np.max(np.abs(sol["lam"] - lam_ref)) / max(1.0, np.max(np.abs(lam_ref))) <= 1e-6
    E = kkt_error(m, sol["y"], sol["lam"], sol["omega_d"], sol["zL"], sol["zU"])
    assert E["max"] <= 1e-8, E
    q = _problem(w)
    import time
    t = time.perf_counter()
    q.autotune(reps=2)
    assert time.perf_counter() - t < 0.5
    r2 = q.solve(warm=False)
    assert r2.iters == r.iters and np.array_equal(q.solution()["y"], sol["y"])
