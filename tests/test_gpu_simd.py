"""Models of the stage-pattern front end (eq. 3; family
NMPC_FAMILY_STAGE_MODEL) on the GPU against the oracle's hand-written models,
through the C ABI: the generated kernels' values and derivatives, Lifted-KKT
and HyKKT solves (certified, then compared entry by entry after each side
tightens its own point on the final barrier problem), sensitivities (the
linear-quadratic model's state rows hold the previous states through a
matrix, so its x0 sensitivities go through that matrix; against the Riccati
gain too), the shifted warm start, a batch mixing generated and hand-written
families, and the re-solve loop of the listing in Section 3.3."""
import numpy as np
import pytest

from oracle.adjoint import sensitivities
from oracle.hykkt import HyKKTIPM
from oracle.ipm import IPMOptions, IPMState, LiftedIPM
from oracle.kkt import kkt_error
from oracle.lq import LQOCP
from oracle.reflux import RefluxColumnOCP
from oracle.riccati import riccati_gains
from oracle.toy import ToyOCP
from paper_2606_04725_amd import capi, simd
from paper_2606_04725_amd import nmpc as N
from paper_2606_04725_amd import simd_models as SM
from plate_parity import PARITY_TOL, TIGHT_TOL, note, rel_dev
from workloads import random_lq, reflux_workload

pytestmark = pytest.mark.gpu

LQ_SHAPE = dict(nx=4, nu=2, H=20, seed=0)


def _toy(traj_shift=0.4, y0=0.7):
    m = ToyOCP()
    traj = np.sin(m.t + traj_shift)
    m.set_parameters(y0=y0, traj=traj)
    g = simd.compile(SM.toy_model())
    p = N.Problem(N.stage_model_structure(g, m.H, m.dt))
    p.analyze()
    p.set_parameters([y0], traj=traj, u_prev=[2.0])
    return m, p


def _lq():
    A, B, Q, R, x0, xs = random_lq(**LQ_SHAPE)
    H = LQ_SHAPE["H"]
    m = LQOCP(A, B, Q, R, H, xs=xs)
    m.set_parameters(x0=x0)
    g = simd.compile(SM.lq_model(A, B, Q, R))
    p = N.Problem(N.stage_model_structure(g, H, 1.0))
    p.analyze()
    p.set_parameters(x0, setpoint=xs, u_prev=np.zeros(2))
    return m, p, (A, B, Q, R, x0, xs)


def _reflux(H, model="stage"):
    w = reflux_workload(H=H)
    m = RefluxColumnOCP(H=H)
    m.set_parameters(x0=w.x0, setpoint=[w.xbar, w.ubar], u_prev=[w.u_prev0])
    make = SM.reflux_model if model == "stage" else SM.reflux_pattern_model
    g = simd.compile(make(N=w.N, Nf=w.Nf, D=w.D, F=w.F, alpha=w.alpha, xf=w.xf, Ac=w.Ac, At=w.At, Ar=w.Ar,
                          w_u=w.w_u))
    p = N.Problem(N.stage_model_structure(g, H, w.dt))
    p.analyze()
    p.set_parameters(w.x0, setpoint=[w.xbar, w.ubar], u_prev=[w.u_prev0])
    return w, m, p


def _column(kind, seed=0, H=None, model="stage"):
    """The workload column written with the front end (as a stage model or
    as index-data patterns), and the oracle's."""
    from oracle.distillation import DistillationOCP
    from workloads import distillation_workload
    w = distillation_workload(kind, seed) if H is None else distillation_workload(kind, seed, H=H)
    m = DistillationOCP.from_workload(w)
    m.set_parameters(x0=w.x0, zF=w.zF(0), u_prev=w.u_prev0)
    make = SM.distillation_model if model == "stage" else SM.distillation_pattern_model
    g = simd.compile(make(w.N, w.alpha, F=w.F, rho=w.rho, x_lo=w.x_lo, x_hi=w.x_hi, u_lo=w.u_lo, u_hi=w.u_hi))
    p = N.Problem(N.stage_model_structure(g, w.H, w.dt))
    p.analyze()
    p.set_parameters(w.x0, setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(0), u_prev=w.u_prev0)
    return w, m, p


def _case(name):
    if name == "toy":
        return _toy()
    if name == "lq":
        return _lq()[:2]
    if name == "column":
        return _column("small")[1:]
    if name == "column_pattern":
        return _column("small", model="pattern")[1:]
    if name == "reflux_pattern":
        return _reflux(10, "pattern")[1:]
    return _reflux(10)[1:]


@pytest.mark.parametrize("name", ["toy", "lq", "reflux", "column", "column_pattern", "reflux_pattern"])
def test_generated_eval_matches_oracle(name):
    import scipy.sparse as sps
    note(f"stage model eval {name}")
    m, p = _case(name)
    rng = np.random.default_rng(5)
    y = m.initial_guess() + 0.05 * rng.normal(size=m.n)
    lam, lam_d = rng.normal(size=m.m_c), rng.normal(size=m.m_d)
    out = p.eval(y, lam, lam_d)
    pat = p.patterns()
    assert abs(out["f"] - m.f(y)) <= 1e-13 * max(1.0, abs(m.f(y)))
    assert rel_dev(out["grad"], m.grad(y)) <= 1e-13
    assert rel_dev(out["c"], m.cons_c(y)) <= 1e-13
    if m.m_d:
        assert rel_dev(out["d"], m.cons_d(y)) <= 1e-13
    J = sps.vstack([m.jac_c(y), m.jac_d(y)]).tocsr() if m.m_d else m.jac_c(y).tocsr()
    assert rel_dev(out["j_vals"], np.asarray(J[pat["j_rows"], pat["j_cols"]]).ravel()) <= 1e-13
    W = m.hess(y, lam, lam_d).tocsr()
    assert rel_dev(out["w_vals"], np.asarray(W[pat["w_rows"], pat["w_cols"]]).ravel()) <= 1e-13


def _compare(ipm, sol, st, tol=1e-6):
    lam, nu = ipm.multipliers(st)
    for key, got, want in (("y", sol["y"], st.y), ("lam", sol["lam"], lam), ("nu", sol["omega_d"], nu),
                           ("zL", sol["zL"], st.zL), ("zU", sol["zU"], st.zU)):
        if len(want) == 0:
            continue
        d = rel_dev(got, want)
        note(f"tightened {key}: {d:.2e}")
        assert d <= tol, (key, d)


@pytest.mark.parametrize("name,route", [("toy", "lifted"), ("lq", "lifted"), ("reflux", "lifted"),
                                        ("column", "lifted"), ("toy", "hykkt"), ("lq", "hykkt"),
                                        ("column", "hykkt")])
def test_generated_solve_matches_oracle(name, route):
    note(f"stage model solve {name} {route}")
    m, p = _case(name)
    hyk = route == "hykkt"
    o = IPMOptions(tol=PARITY_TOL)
    ipm = HyKKTIPM(m, o) if hyk else LiftedIPM(m, o)
    ref = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
    assert ref.status == 0
    kw = dict(kkt=capi.NMPC_KKT_HYKKT) if hyk else {}
    r = p.solve(warm=False, options=N.default_options(tol=PARITY_TOL, **kw))
    note(f"iterations gpu {r.iters} oracle {ref.iters}; mu gpu {r.mu:.2e} oracle {ref.mu:.2e}")
    assert r.status == 0
    assert r.mu == ipm.o.mu_min and ref.mu == ipm.o.mu_min
    assert abs(r.iters - ref.iters) <= 2
    sol = p.solution()
    e = kkt_error(m, sol["y"], sol["lam"], sol["omega_d"], sol["zL"], sol["zU"])
    assert e["max"] <= 1e-8, e
    rt = p.solve(warm=True, options=N.default_options(fixed_mu=1, tol=TIGHT_TOL, mu0_warm=r.mu, max_iter=30, **kw))
    assert rt.status == 0
    ref_t = ipm.solve(ref.state, ref.mu, fixed_mu=True, tol=TIGHT_TOL)
    assert ref_t.status == 0
    _compare(ipm, p.solution(), ref_t.state)


@pytest.mark.parametrize("model", ["stage", "pattern"])
def test_generated_case_study_equals_the_hand_written_family(model):
    """The case-study column written with the front end (as a stage model,
    or as index-data patterns with algebraic rows and guess patterns) and the
    library's REFLUX_COLUMN family solve the same problem at the full horizon
    (90 stages): same iteration count, points equal to 1e-9 after
    tightening."""
    note(f"generated ({model}) vs hand-written case-study column, H=90")
    w, m, pg = _reflux(90, model)
    ph = N.Problem(N.reflux_structure(90))
    ph.analyze()
    ph.set_parameters(w.x0, setpoint=[w.xbar, w.ubar], u_prev=[w.u_prev0])
    out = []
    for p in (pg, ph):
        r = p.solve(warm=False)
        assert r.status == 0
        rt = p.solve(warm=True, options=N.default_options(fixed_mu=1, tol=TIGHT_TOL, mu0_warm=r.mu, max_iter=30))
        assert rt.status == 0
        out.append((r.iters, p.solution()))
    note(f"iterations generated {out[0][0]} hand-written {out[1][0]}")
    assert abs(out[0][0] - out[1][0]) <= 1
    for key in ("y", "lam", "zL", "zU"):
        d = rel_dev(out[0][1][key], out[1][1][key])
        note(f"{key}: {d:.2e}")
        assert d <= 1e-9, (key, d)
    sol = out[0][1]
    assert kkt_error(m, sol["y"], sol["lam"], sol["omega_d"], sol["zL"], sol["zU"])["max"] <= 1e-8


@pytest.mark.parametrize("model", ["stage", "pattern"])
def test_generated_workload_column_equals_the_hand_written_family(model):
    """The headline workload (40 trays, horizon 100) written with the front
    end (as a stage model, or as index-data patterns) and the library's
    DISTILLATION family, over a cold solve and five warm re-solves of the
    workload's closed loop at the default options (both fed the hand-written
    side's first stage): equal iteration counts, returned points within 1e-7
    of each other (both stop inside the default tolerance's ball; their model
    values differ only by rounding order)."""
    note(f"generated ({model}) vs hand-written workload column, 40 trays, H=100")
    w, m, pg = _column("medium", model=model)
    ph = N.Problem(N.distillation_structure(w.N, w.H, w.dt, w.alpha, F=w.F, rho=w.rho))
    ph.analyze()
    sp = [w.xD_sp, w.xB_sp]
    x0, up = w.x0, w.u_prev0
    for k in range(6):
        res = []
        for p in (pg, ph):
            p.set_parameters(x0, setpoint=sp, traj=w.zF(k), u_prev=up)
            r = p.solve(warm=k > 0)
            assert r.status == 0
            res.append((r.iters, p.solution()))
        note(f"solve {k}: iterations generated {res[0][0]} hand-written {res[1][0]}")
        assert res[0][0] == res[1][0]
        for key in ("y", "lam", "omega_d", "zL", "zU"):
            d = rel_dev(res[0][1][key], res[1][1][key])
            assert d <= 1e-7, (k, key, d)
        up, x1 = res[1][1]["u1"], res[1][1]["x1"]
        x0 = w.next_measurement(x1, k)


@pytest.mark.parametrize("model", ["stage", "pattern"])
def test_column_model_sensitivities_match_oracle(model):
    note(f"{model} model sensitivities: workload column (x0, setpoint, traj, u_prev)")
    w, m, p = _column("small", seed=2, model=model)
    ipm, st = _solved(m, p)
    sens = sensitivities(ipm, st)
    su, so = np.array([0.4, -1.1]), 0.3
    rc, g = p.adjoint(su, so)
    assert rc == 0
    for key, rk in (("x0", "x0"), ("setpoint", "setpoint"), ("traj", "zF"), ("u_prev", "u_prev")):
        d = rel_dev(g[key], su @ sens[rk]["du1"] + so * sens[rk]["df"])
        note(f"{key}: {d:.2e}")
        assert d <= 1e-6, (key, d)


def _solved(m, p):
    ipm = LiftedIPM(m)
    res = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
    assert res.status == 0
    st = res.state
    p.set_iterate(st.y, st.s, st.omega, st.beta, st.zL, st.zU)
    return ipm, st


def test_toy_sensitivities_match_oracle():
    note("stage model sensitivities: toy (y0, trajectory)")
    m, p = _toy()
    ipm, st = _solved(m, p)
    sens = sensitivities(ipm, st)
    su, so = np.array([1.3]), 0.4
    rc, g = p.adjoint(su, so)
    assert rc == 0
    for key, rk in (("x0", "y0"), ("traj", "traj")):
        want = su @ sens[rk]["du1"] + so * sens[rk]["df"]
        d = rel_dev(g[key], want)
        note(f"{key}: {d:.2e}")
        assert d <= 1e-6, (key, d)
    assert g["setpoint"].size == 0 and np.all(g["u_prev"] == 0.0)
    rc, J = p.jacobian_u1_x0()
    assert rc == 0 and rel_dev(J, sens["y0"]["du1"]) <= 1e-6


def test_lq_sensitivities_through_the_state_matrix():
    """d u1 / d x0 of the linear-quadratic model: against the oracle's
    sensitivity solve and against the Riccati gain -K_1 (to the lifting's
    O(gamma) relaxation); the allocation-free Jacobian equals the other."""
    note("stage model sensitivities: LQ (x0 through A)")
    m, p, (A, B, Q, R, x0, xs) = _lq()
    ipm, st = _solved(m, p)
    sens = sensitivities(ipm, st)
    rc, J = p.jacobian_u1_x0()
    assert rc == 0
    d = rel_dev(J, sens["x0"]["du1"])
    note(f"jacobian vs oracle: {d:.2e}")
    assert d <= 1e-6
    K, _ = riccati_gains(A, B, Q, R, LQ_SHAPE["H"], xs)
    assert np.allclose(J, -K[1], rtol=1e-5, atol=2e-6)
    su, so = np.array([0.5, -1.0]), 0.25
    rc, g = p.adjoint(su, so)
    assert rc == 0
    for key, rk in (("x0", "x0"), ("setpoint", "xs")):
        want = su @ sens[rk]["du1"] + so * sens[rk]["df"]
        d = rel_dev(g[key], want)
        note(f"{key}: {d:.2e}")
        assert d <= 1e-6, (key, d)
    import ctypes as C
    import torch
    jd = torch.zeros((p.nu, p.nx), dtype=torch.float64, device="cuda")
    rc = N._check(capi.lib().nmpc_jacobian_u1_x0_noalloc(p._h, C.c_void_p(jd.data_ptr()), None))
    torch.cuda.synchronize()
    assert rc == 0
    assert np.array_equal(jd.cpu().numpy(), J)


@pytest.mark.parametrize("model", ["stage", "pattern"])
def test_reflux_model_sensitivities_match_oracle(model):
    note(f"{model} model sensitivities: case-study column (x0, setpoint)")
    w, m, p = _reflux(10, model)
    ipm, st = _solved(m, p)
    sens = sensitivities(ipm, st)
    su, so = np.array([0.8]), 0.3
    rc, g = p.adjoint(su, so)
    assert rc == 0
    for key in ("x0", "setpoint"):
        want = su @ sens[key]["du1"] + so * sens[key]["df"]
        d = rel_dev(g[key], want)
        note(f"{key}: {d:.2e}")
        assert d <= 1e-6, (key, d)


@pytest.mark.parametrize("which", ["generated", "hand-written"])
def test_shift_of_the_case_study_matches_oracle_bit_for_bit(which):
    """2 N + 3 equality rows per stage move together (index work: exact)."""
    from oracle.nmpc import shift_state
    note(f"shifted warm start: case-study column, {which}")
    w, m, p = _reflux(6)
    if which == "hand-written":
        p = N.Problem(N.reflux_structure(6))
        p.analyze()
        p.set_parameters(w.x0, setpoint=[w.xbar, w.ubar], u_prev=[w.u_prev0])
    rng = np.random.default_rng(2)
    ml = 2 * m.m_c + m.m_d
    st = IPMState(rng.uniform(0.1, 0.9, m.n), *(rng.uniform(0.5, 2.0, ml) for _ in range(3)),
                  rng.uniform(0.1, 1.0, m.n), rng.uniform(0.1, 1.0, m.n))
    p.set_iterate(st.y, st.s, st.omega, st.beta, st.zL, st.zU)
    r = p.solve(warm="shift", options=N.default_options(max_iter=0))
    assert r.iters == 0
    got, want = p.get_iterate(), shift_state(m, st)
    for key in ("y", "s", "omega", "beta", "zL", "zU"):
        assert np.array_equal(got[key], getattr(want, key)), key


def test_batch_mixing_generated_and_hand_written_families():
    """One batch holding the toy model, the LQ model and a distillation column:
    every instance's result is the one of its own solve, bit for bit."""
    from workloads import distillation_workload
    note("batch: toy + LQ + distillation column")

    def make():
        _, pt = _toy()
        _, pl, _ = _lq()
        w = distillation_workload("small", 0)
        pd = N.Problem(N.distillation_structure(w.N, w.H, w.dt, w.alpha, F=w.F, rho=w.rho))
        pd.analyze()
        pd.set_parameters(w.x0, setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(0), u_prev=w.u_prev0)
        return [pt, pl, pd]

    batched, single = make(), make()
    b = N.Batch(batched)
    rc, res = b.solve(warm=False)
    assert rc == 0, [r.status for r in res]
    for i, (pb, ps) in enumerate(zip(batched, single)):
        r1 = ps.solve(warm=False)
        assert r1.status == 0 and res[i].iters == r1.iters, i
        sb, ss = pb.solution(), ps.solution()
        for key in ("y", "lam", "zL", "zU"):
            assert np.array_equal(sb[key], ss[key]), (i, key)
    b.close()


def test_resolve_loop_of_the_listing():
    """The re-solve loop of the listing in Section 3.3: solve, apply the
    first control to the explicit-Euler plant of the listing (dt 1), update
    y0 and the trajectory sin(t + tk), re-solve warm.  Each GPU solve is
    certified for its parameters and its first control equals the oracle's
    (both sides start every step from the same measurement)."""
    note("re-solve loop of the listing, 6 steps")
    m = ToyOCP()
    g = simd.compile(SM.toy_model())
    p = N.Problem(N.stage_model_structure(g, m.H, m.dt))
    p.analyze()
    ipm = LiftedIPM(m, IPMOptions(tol=PARITY_TOL))
    y_meas, st = 1.0, None
    for tk in range(6):
        traj = np.sin(m.t + tk)
        m.set_parameters(y0=y_meas, traj=traj)
        p.set_parameters([y_meas], traj=traj, u_prev=[2.0])
        ref = (ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold) if st is None
               else ipm.solve(st, ipm.o.mu0_warm))
        r = p.solve(warm=tk > 0, options=N.default_options(tol=PARITY_TOL))
        note(f"step {tk}: iterations gpu {r.iters} oracle {ref.iters}")
        assert r.status == 0 and ref.status == 0 and abs(r.iters - ref.iters) <= 2
        sol = p.solution()
        assert kkt_error(m, sol["y"], sol["lam"], sol["omega_d"], sol["zL"], sol["zU"])["max"] <= 1e-8
        assert p.solve(warm=True, options=N.default_options(fixed_mu=1, tol=TIGHT_TOL, mu0_warm=r.mu,
                                                             max_iter=30)).status == 0
        ref_t = ipm.solve(ref.state, ref.mu, fixed_mu=True, tol=TIGHT_TOL)
        assert ref_t.status == 0
        st = ref_t.state
        u1_gpu, _ = p.first_stage()
        u1 = m.u1(st.y)
        assert abs(u1_gpu[0] - u1[0]) <= 1e-6 * max(1.0, abs(u1[0]))
        y_meas = y_meas + 1.0 * (4.0 * np.sin(u1[0]) - y_meas ** 3)
