"""The workload plate written with index-data patterns (one stencil row
pattern, one tracking pattern; eq. 3's repeated pattern over the grid) on the
GPU, through the C ABI: model values and derivatives against the oracle's
transcription (oracle/plate.py), whole solves and sensitivities against the
oracle, and at the 32 x 32 x 50 workload size the condensed matrix entry by
entry and the solve against the library's hand-written plate family."""
import numpy as np
import pytest

from oracle.adjoint import sensitivities
from oracle.ipm import IPMOptions, LiftedIPM
from oracle.kkt import kkt_error
from oracle.plate import PlateOCP
from paper_2606_04725_amd import nmpc as N
from paper_2606_04725_amd import simd
from paper_2606_04725_amd import simd_models as SM
from plate_parity import PARITY_TOL, close, note, rel_dev, solve_pair, tighten_gpu, tighten_ref
from workloads import plate_workload

pytestmark = pytest.mark.gpu


def _pattern_problem(w, m):
    g = simd.compile(SM.plate_pattern_model(w.G))
    p = N.Problem(N.stage_model_structure(g, w.H, w.dt))
    p.analyze()
    p.set_parameters(w.T0, setpoint=w.target, u_prev=m.u_prev)
    return p


def _pair(G, H, seed=0):
    w = plate_workload("large", seed, G=G, H=H)
    m = PlateOCP.from_workload(w)
    return w, m, _pattern_problem(w, m)


def test_pattern_plate_eval_matches_oracle():
    note("pattern plate eval G=8 H=3")
    w, m, p = _pair(8, 3)
    rng = np.random.default_rng(1)
    y = rng.uniform(0.0, 1.0, m.n)
    lam = rng.normal(size=m.m_c)
    for _ in range(2):           # the scratch keeps the first call's values: the second must not see them
        out = p.eval(y, lam, np.zeros(0))
        pat = p.patterns()
        assert abs(out["f"] - m.f(y)) <= 1e-13 * max(1.0, abs(m.f(y)))
        assert close(out["grad"], m.grad(y), 1e-13)
        assert close(out["c"], m.cons_c(y), 1e-13)
        J = m.jac_c(y).tocsr()
        assert close(out["j_vals"], np.asarray(J[pat["j_rows"], pat["j_cols"]]).ravel(), 1e-13)
        W = m.hess(y, lam, np.zeros(0)).tocsr()
        assert close(out["w_vals"], np.asarray(W[pat["w_rows"], pat["w_cols"]]).ravel(), 1e-13)
        y = rng.uniform(0.0, 1.0, m.n)
        lam = rng.normal(size=m.m_c)


@pytest.mark.parametrize("G,H,seed", [(8, 5, 1), (16, 10, 0)])
def test_pattern_plate_solve_matches_oracle(G, H, seed):
    """Cold solve, one plant step, warm re-solve; each compared with the
    oracle after both tighten on the final barrier problem."""
    note(f"pattern plate solve G={G} H={H} seed={seed}")
    w, m, p = _pair(G, H, seed)
    ipm = LiftedIPM(m, IPMOptions(tol=PARITY_TOL))
    ref = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
    assert ref.status == 0
    ref_t = solve_pair(m, p, ipm, ref, warm=False)
    x1 = m.step(m.x0, m.u1(ref_t.state.y))
    m.set_parameters(x0=x1)
    p.set_parameters(x1)
    ref2 = ipm.solve(ref_t.state, ipm.o.mu0_warm)
    assert ref2.status == 0
    solve_pair(m, p, ipm, ref2, warm=True)


def test_pattern_plate_adjoint_matches_oracle():
    """Sensitivities to the measured field and to the target field at the
    oracle's tightened point (placed on the GPU with set_iterate)."""
    note("pattern plate adjoint G=8 H=3")
    w, m, p = _pair(8, 3)
    ipm = LiftedIPM(m, IPMOptions(tol=PARITY_TOL))
    ref = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
    assert ref.status == 0
    st = tighten_ref(ipm, ref).state
    sens = sensitivities(ipm, st)
    rng = np.random.default_rng(4)
    su, so = rng.normal(size=16), float(rng.normal())
    p.set_iterate(st.y, st.s, st.omega, st.beta, st.zL, st.zU)
    rc, g = p.adjoint(su, so)
    assert rc == 0
    for key in ("x0", "setpoint"):
        d = rel_dev(g[key], su @ sens[key]["du1"] + so * sens[key]["df"])
        note(f"{key}: {d:.2e}")
        assert d <= 1e-6, (key, d)
    assert np.all(g["u_prev"] == 0.0)
    rc, J = p.jacobian_u1_x0()
    assert rc == 0 and close(J, sens["x0"]["du1"], 1e-6)


def test_pattern_plate_workload_size_matches_hand_written_family():
    """32 x 32 grid, horizon 50 (n = 52,000): at one point the generated and
    the hand-written kernels give the same condensed matrix (entries keyed by
    position; the two analyses order columns differently); a cold solve of
    each converges (optimality error of the original problem <= 1e-8 by the
    oracle's evaluator) and, tightened on the final barrier problem, the two
    agree to 1e-6."""
    note("pattern plate vs hand-written family, G=32 H=50")
    w = plate_workload("large", 0)
    m = PlateOCP.from_workload(w)
    pg = _pattern_problem(w, m)
    ph = N.Problem(N.plate_structure(w.G, w.H, w.dt, t_hi=w.T_hi, c_lo=w.u_lo, c_hi=w.u_hi))
    ph.analyze()
    ph.set_parameters(w.T0, setpoint=w.target, u_prev=m.u_prev)
    ipm = LiftedIPM(m)
    st = ipm.cold_start(m.initial_guess(), 0.1)
    st.omega = np.random.default_rng(5).normal(scale=0.5, size=ipm.ml)
    kk = []
    for p in (pg, ph):
        p.set_iterate(st.y, st.s, st.omega, st.beta, st.zL, st.zU)
        kv, rhs = p.assemble(0.1)
        pat = p.patterns()
        order = np.lexsort((pat["k_cols"], pat["k_rows"]))
        kk.append((pat["k_rows"][order], pat["k_cols"][order], kv[order], rhs))
    assert np.array_equal(kk[0][0], kk[1][0]) and np.array_equal(kk[0][1], kk[1][1])
    assert close(kk[0][2], kk[1][2], 1e-12)
    assert close(kk[0][3], kk[1][3], 1e-12)
    res = []
    for p in (pg, ph):
        r = p.solve(warm=False, options=N.default_options(tol=PARITY_TOL))
        assert r.status == 0, r.status
        sol = p.solution()
        e = kkt_error(m, sol["y"], sol["lam"], np.zeros(0), sol["zL"], sol["zU"])
        assert e["max"] <= 1e-8, e
        tighten_gpu(p, r.mu)
        res.append((r.iters, p.solution()))
    note(f"iterations generated {res[0][0]} hand-written {res[1][0]}")
    assert abs(res[0][0] - res[1][0]) <= 2
    for key in ("y", "lam", "zL", "zU"):
        d = rel_dev(res[0][1][key], res[1][1][key])
        note(f"tightened {key}: {d:.2e}")
        assert d <= 1e-6, (key, d)


def test_pattern_batch_equals_one_by_one():
    """One batch holding two instances of the pattern plate (different
    targets and fields: each has its own scratch) and the hand-written plate:
    every instance's iterations and solution are those of its own solve, bit
    for bit, over a cold solve and a warm re-solve."""
    note("batch: pattern plate x 2 + hand-written plate, G=8 H=5")

    def make():
        out = []
        for seed in (0, 1):
            w = plate_workload("large", seed, G=8, H=5)
            out.append((w, _pattern_problem(w, PlateOCP.from_workload(w))))
        w = plate_workload("large", 2, G=8, H=5)
        p = N.Problem(N.plate_structure(8, 5, w.dt, t_hi=w.T_hi, c_lo=w.u_lo, c_hi=w.u_hi))
        p.analyze()
        p.set_parameters(w.T0, setpoint=w.target, u_prev=PlateOCP.from_workload(w).u_prev)
        out.append((w, p))
        return out

    batched, single = make(), make()
    b = N.Batch([p for _, p in batched])
    for k in range(2):
        rc, res = b.solve(warm=k > 0)
        assert rc == 0, [r.status for r in res]
        for i, ((w, pb), (_, ps)) in enumerate(zip(batched, single)):
            r1 = ps.solve(warm=k > 0)
            assert r1.status == 0 and res[i].iters == r1.iters, (k, i, res[i].iters, r1.iters)
            sb, ss = pb.solution(), ps.solution()
            for key in ("y", "lam", "zL", "zU"):
                assert np.array_equal(sb[key], ss[key]), (k, i, key)
        for (w, pb), (_, ps) in zip(batched, single):
            u1, x1 = ps.first_stage()
            for p in (pb, ps):
                p.set_parameters(x1, setpoint=w.target, u_prev=u1)
    b.close()


def test_every_row_kind_generated_eval_matches_the_derivation():
    """A model with state, algebraic and inequality row patterns: the
    generated kernels' values, Jacobian and Hessian entries (keyed by
    position), gradient and objective equal the host evaluation of the same
    derived expressions (tests/simd_eval.py), at 1e-13."""
    from simd_eval import expand_patterns
    note("pattern model with algebraic and inequality rows: eval")
    g = simd.compile(SM.row_kinds_model())
    H, dt = 3, 0.2
    p = N.Problem(N.stage_model_structure(g, H, dt))
    p.analyze()
    rng = np.random.default_rng(9)
    x0 = rng.normal(size=2)
    p.set_parameters(x0, u_prev=[0.3, -0.2])
    y = rng.normal(size=H * 5)
    lam, lam_d = rng.normal(size=H * 3), rng.uniform(0.1, 1.0, size=H * 2)
    out = p.eval(y, lam, lam_d)
    ref = expand_patterns(g, y, H, x0, dt, lam=lam, lam_d=lam_d)
    assert abs(out["f"] - ref["f"]) <= 1e-13 * max(1.0, abs(ref["f"]))
    assert close(out["grad"], ref["grad"], 1e-13)
    assert close(out["c"], ref["c"], 1e-13)
    assert close(out["d"], ref["d"], 1e-13)
    pat = p.patterns()
    jref = dict(zip(zip(ref["jr"].tolist(), ref["jc"].tolist()), ref["jv"]))
    assert len(jref) == len(pat["j_rows"])
    assert close(out["j_vals"], [jref[(r, c)] for r, c in zip(pat["j_rows"].tolist(), pat["j_cols"].tolist())],
                 1e-13)
    wref = dict(zip(zip(ref["wr"].tolist(), ref["wc"].tolist()), ref["wv"]))
    assert close(out["w_vals"], [wref[(r, c)] for r, c in zip(pat["w_rows"].tolist(), pat["w_cols"].tolist())],
                 1e-13)


def test_pattern_plate_closed_loop_on_the_device_equals_the_host_loop():
    """Algorithm 1 on the device (nmpc_closed_loop_dev: the parameter update
    and the first passes of each re-solve in one captured graph, the
    evaluation and the summing kernel inside it) with the pattern plate:
    the applied controls, predicted fields, iteration counts and final
    iterate equal the host-driven loop bit for bit."""
    import torch
    note("closed loop on the device, pattern plate G=8 H=5, 6 steps")
    steps = 6

    def make():
        w = plate_workload("large", 0, G=8, H=5)
        p = _pattern_problem(w, PlateOCP.from_workload(w))
        assert p.solve(warm=False).status == 0
        return w, p

    (w, ph), (_, pd) = make(), make()
    us, xs, iters = [], [], 0
    for k in range(steps):
        u1, x1 = ph.first_stage()
        us.append(u1)
        xs.append(x1)
        ph.set_parameters(x1, setpoint=w.target, u_prev=u1)
        r = ph.solve(warm=True)
        assert r.status == 0
        iters += r.iters
    u_out = torch.zeros((steps, pd.nu), dtype=torch.float64, device="cuda")
    x_out = torch.zeros((steps, pd.nx), dtype=torch.float64, device="cuda")
    rc, done, it = pd.closed_loop_dev(steps, u_out=u_out.data_ptr(), x_out=x_out.data_ptr(), passes_per_step=2)
    torch.cuda.synchronize()
    assert rc == 0 and done == steps and it == iters
    assert np.array_equal(u_out.cpu().numpy(), np.array(us))
    assert np.array_equal(x_out.cpu().numpy(), np.array(xs))
    for key in ("y", "lam", "zL", "zU"):
        assert np.array_equal(ph.solution()[key], pd.solution()[key]), key
