"""The heated-plate case study of Section 4.2 (Table 2), written with the
stage-pattern front end, on the GPU against the oracle's transcription
(oracle/plate_case.py), through the C ABI: model values and derivatives on
the 21 x 21 grid, the first NMPC solve (certified, then compared entry by
entry after each side tightens its point on the final barrier problem), the
sensitivities (the measured field enters the first stage's rows with the row
scale as coefficient, so they go through the state rows' matrix), and the
closed loop's first steps with each side fed the same measurement.  The
model values, the first solve and the sensitivities are also checked for the
same plate written as index-data patterns (simd_models.plate_case_pattern_model)."""
import numpy as np
import pytest

from oracle.adjoint import sensitivities
from oracle.ipm import IPMOptions, LiftedIPM
from oracle.kkt import kkt_error
from oracle.plate_case import PlateCaseOCP
from paper_2606_04725_amd import nmpc as N
from paper_2606_04725_amd import simd
from paper_2606_04725_amd import simd_models as SM
from plate_parity import PARITY_TOL, TIGHT_TOL, note, rel_dev
from workloads import plate_case_workload

pytestmark = pytest.mark.gpu


def _pair(k=0, model="stage"):
    w = plate_case_workload()
    m = PlateCaseOCP(H=w.H, dt=w.dt, n=w.n, alpha=w.alpha, Tb=w.Tb, loss=w.loss, rho=w.rho, Q_lo=w.Q_lo,
                     q_scale=w.q_scale)
    x0, up = np.full(m.nx, w.T0), np.array([w.Q_prev0 / w.q_scale])
    m.set_parameters(x0=x0, traj=w.traj(k), u_prev=up)
    make = SM.plate_case_model if model == "stage" else SM.plate_case_pattern_model
    g = simd.compile(make(n=w.n, alpha=w.alpha, Tb=w.Tb, loss=w.loss, rho=w.rho, Q_lo=w.Q_lo,
                          q_scale=w.q_scale, dt=w.dt))
    p = N.Problem(N.stage_model_structure(g, w.H, w.dt))
    p.analyze()
    p.set_parameters(x0, traj=w.traj(k), u_prev=up)
    return w, m, p


@pytest.mark.parametrize("model", ["stage", "pattern"])
def test_plate_case_eval_matches_oracle(model):
    note(f"plate case study eval, 21 x 21, H 12, {model} model")
    w, m, p = _pair(model=model)
    rng = np.random.default_rng(4)
    y = m.initial_guess() + rng.normal(size=m.n)
    y[m.nx::m.ns] = rng.uniform(0.3, 1.5, m.H)
    lam = rng.normal(size=m.m_c)
    out = p.eval(y, lam, np.zeros(0))
    pat = p.patterns()
    assert abs(out["f"] - m.f(y)) <= 1e-13 * max(1.0, abs(m.f(y)))
    assert rel_dev(out["grad"], m.grad(y)) <= 1e-13
    assert rel_dev(out["c"], m.cons_c(y)) <= 1e-13
    J = m.jac_c(y).tocsr()
    assert rel_dev(out["j_vals"], np.asarray(J[pat["j_rows"], pat["j_cols"]]).ravel()) <= 1e-13
    W = m.hess(y, lam, np.zeros(0)).tocsr()
    assert rel_dev(out["w_vals"], np.asarray(W[pat["w_rows"], pat["w_cols"]]).ravel()) <= 1e-13


def _compare(ipm, sol, st, tol=1e-6):
    lam, _ = ipm.multipliers(st)
    for key, got, want in (("y", sol["y"], st.y), ("lam", sol["lam"], lam), ("zL", sol["zL"], st.zL)):
        d = rel_dev(got, want)
        note(f"tightened {key}: {d:.2e}")
        assert d <= tol, (key, d)


@pytest.mark.parametrize("model", ["stage", "pattern"])
def test_plate_case_first_solve_matches_oracle(model):
    note(f"plate case study first solve, {model} model")
    w, m, p = _pair(model=model)
    ipm = LiftedIPM(m, IPMOptions(tol=PARITY_TOL))
    ref = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
    assert ref.status == 0
    r = p.solve(warm=False, options=N.default_options(tol=PARITY_TOL))
    note(f"iterations gpu {r.iters} oracle {ref.iters}; mu gpu {r.mu:.2e} oracle {ref.mu:.2e}")
    assert r.status == 0 and r.mu == ipm.o.mu_min and ref.mu == ipm.o.mu_min
    assert abs(r.iters - ref.iters) <= 2
    sol = p.solution()
    assert kkt_error(m, sol["y"], sol["lam"], sol["omega_d"], sol["zL"], sol["zU"])["max"] <= 1e-8
    assert p.solve(warm=True, options=N.default_options(fixed_mu=1, tol=TIGHT_TOL, mu0_warm=r.mu,
                                                         max_iter=30)).status == 0
    ref_t = ipm.solve(ref.state, ref.mu, fixed_mu=True, tol=TIGHT_TOL)
    assert ref_t.status == 0
    _compare(ipm, p.solution(), ref_t.state)


@pytest.mark.parametrize("model", ["stage", "pattern"])
def test_plate_case_sensitivities_match_oracle(model):
    """At a constant setpoint over the horizon.  (A setpoint step inside the
    horizon drives the lifted weights of the rows around it to 1e16-1e17 at
    mu_min: the condensed matrix at the solution is then numerically
    indefinite and the sensitivity solve reports NMPC_REG_FAIL.)"""
    note(f"plate case study sensitivities (x0 through the row scale, trajectory), {model} model")
    w, m, p = _pair(model=model)
    m.set_parameters(traj=np.full(w.H, 58.0))
    p.set_parameters(m.x0, traj=np.full(w.H, 58.0), u_prev=m.u_prev)
    ipm = LiftedIPM(m)
    res = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
    assert res.status == 0
    st = res.state
    p.set_iterate(st.y, st.s, st.omega, st.beta, st.zL, st.zU)
    sens = sensitivities(ipm, st)
    su, so = np.array([1.0]), 1e-3
    rc, g = p.adjoint(su, so)
    assert rc == 0
    for key in ("x0", "traj"):
        d = rel_dev(g[key], su @ sens[key]["du1"] + so * sens[key]["df"])
        note(f"{key}: {d:.2e}")
        assert d <= 1e-6, (key, d)
    rc, J = p.jacobian_u1_x0()
    assert rc == 0 and rel_dev(J, sens["x0"]["du1"]) <= 1e-6


def test_plate_case_closed_loop_matches_oracle():
    """Six NMPC steps across the first setpoint change (t = 0.5 s enters the
    horizon at once; the current setpoint changes at step 7): every GPU solve
    certified, the first input equal to the oracle's after both tighten; the
    plant is the model, each side fed the oracle's predicted field."""
    note("plate case study closed loop, 6 steps")
    w, m, p = _pair()
    ipm = LiftedIPM(m, IPMOptions(tol=PARITY_TOL))
    x0, up, st = np.full(m.nx, w.T0), np.array([w.Q_prev0 / w.q_scale]), None
    for k in range(6):
        m.set_parameters(x0=x0, traj=w.traj(k), u_prev=up)
        p.set_parameters(x0, traj=w.traj(k), u_prev=up)
        ref = (ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold) if st is None
               else ipm.solve(st, ipm.o.mu0_warm))
        r = p.solve(warm=k > 0, options=N.default_options(tol=PARITY_TOL))
        note(f"step {k}: iterations gpu {r.iters} oracle {ref.iters}")
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
        assert abs(u1_gpu[0] - u1[0]) <= 1e-6 * max(1.0, abs(u1[0])), (k, u1_gpu, u1)
        x0, up = m.x1(st.y), u1
