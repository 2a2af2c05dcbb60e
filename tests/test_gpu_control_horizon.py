"""Control horizon (Section 3.1, eqs. 4-5) on the GPU against the oracle,
through the C ABI: the hold rows' values and Jacobian slots, Lifted-KKT and
HyKKT solves (certified, then compared entry by entry after each side
tightens its point on the final barrier problem) and the sensitivities."""
import numpy as np
import pytest

from oracle.adjoint import sensitivities
from oracle.distillation import DistillationOCP
from oracle.hykkt import HyKKTIPM
from oracle.ipm import IPMOptions, LiftedIPM
from oracle.kkt import kkt_error
from paper_2606_04725_amd import capi
from paper_2606_04725_amd import nmpc as N
from plate_parity import PARITY_TOL, TIGHT_TOL, note, rel_dev
from workloads import distillation_workload

pytestmark = pytest.mark.gpu


def _pair(kind, seed, Hc):
    w = distillation_workload(kind, seed, Hc=Hc)
    m = DistillationOCP.from_workload(w)
    m.set_parameters(x0=w.x0, zF=w.zF(0), u_prev=w.u_prev0)
    p = N.Problem(N.distillation_structure(w.N, w.H, w.dt, w.alpha, F=w.F, rho=w.rho, control_horizon=Hc))
    p.analyze()
    p.set_parameters(w.x0, setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(0), u_prev=w.u_prev0)
    assert p.m_c == m.m_c
    return w, m, p


def test_hold_rows_eval():
    note("control horizon eval, small column Hc 5")
    w, m, p = _pair("small", 0, 5)
    rng = np.random.default_rng(2)
    y = rng.uniform(0.1, 0.9, m.n)
    y[m.nx::m.ns] = rng.uniform(0.6, 4.5, m.H)
    y[m.nx + 1::m.ns] = rng.uniform(0.6, 4.5, m.H)
    lam, lam_d = rng.normal(size=m.m_c), rng.normal(size=m.m_d)
    out = p.eval(y, lam, lam_d)
    assert rel_dev(out["c"], m.cons_c(y)) <= 1e-13
    pat = p.patterns()
    J, Jd = m.jac_c(y).tocsr(), m.jac_d(y).tocsr()
    ref = np.array([J[r, c] if r < m.m_c else Jd[r - m.m_c, c] for r, c in zip(pat["j_rows"], pat["j_cols"])])
    assert rel_dev(out["j_vals"], ref) <= 1e-13
    W = m.hess(y, lam, lam_d).tocsr()
    assert rel_dev(out["w_vals"], np.array([W[r, c] for r, c in zip(pat["w_rows"], pat["w_cols"])])) <= 1e-13


@pytest.mark.parametrize("kind,seed,Hc,route", [("small", 0, 5, "lifted"), ("medium", 0, 20, "lifted"),
                                                 ("small", 1, 4, "hykkt")])
def test_held_solve_matches_oracle(kind, seed, Hc, route):
    note(f"control horizon solve {kind} seed {seed} Hc {Hc} {route}")
    w, m, p = _pair(kind, seed, Hc)
    hyk = route == "hykkt"
    ipm = HyKKTIPM(m, IPMOptions(tol=PARITY_TOL)) if hyk else LiftedIPM(m, IPMOptions(tol=PARITY_TOL))
    ref = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
    assert ref.status == 0
    kw = dict(kkt=capi.NMPC_KKT_HYKKT) if hyk else {}
    r = p.solve(warm=False, options=N.default_options(tol=PARITY_TOL, **kw))
    note(f"iterations gpu {r.iters} oracle {ref.iters}; mu gpu {r.mu:.2e} oracle {ref.mu:.2e}")
    assert r.status == 0 and r.mu == ipm.o.mu_min and ref.mu == ipm.o.mu_min
    assert abs(r.iters - ref.iters) <= 2
    sol = p.solution()
    assert kkt_error(m, sol["y"], sol["lam"], sol["omega_d"], sol["zL"], sol["zU"])["max"] <= 1e-8
    U = sol["y"].reshape(m.H, m.ns)[:, m.nx:]
    assert np.max(np.abs(U[Hc:] - U[Hc - 1])) <= 1e-7
    rt = p.solve(warm=True, options=N.default_options(fixed_mu=1, tol=TIGHT_TOL, mu0_warm=r.mu, max_iter=30, **kw))
    assert rt.status == 0
    ref_t = ipm.solve(ref.state, ref.mu, fixed_mu=True, tol=TIGHT_TOL)
    assert ref_t.status == 0
    lam, nu = ipm.multipliers(ref_t.state)
    sol = p.solution()
    for key, got, want in (("y", sol["y"], ref_t.state.y), ("lam", sol["lam"], lam), ("nu", sol["omega_d"], nu),
                           ("zL", sol["zL"], ref_t.state.zL), ("zU", sol["zU"], ref_t.state.zU)):
        d = rel_dev(got, want)
        note(f"tightened {key}: {d:.2e}")
        assert d <= 1e-6, (key, d)


def test_held_sensitivities_match_oracle():
    note("control horizon sensitivities, small column Hc 6")
    w, m, p = _pair("small", 2, 6)
    ipm = LiftedIPM(m)
    res = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
    assert res.status == 0
    st = res.state
    p.set_iterate(st.y, st.s, st.omega, st.beta, st.zL, st.zU)
    sens = sensitivities(ipm, st)
    su, so = np.array([0.4, -1.1]), 0.3
    rc, g = p.adjoint(su, so)
    assert rc == 0
    for key, rk in (("x0", "x0"), ("setpoint", "setpoint"), ("traj", "zF"), ("u_prev", "u_prev")):
        d = rel_dev(g[key], su @ sens[rk]["du1"] + so * sens[rk]["df"])
        assert d <= 1e-6, (key, d)
    rc, J = p.jacobian_u1_x0()
    assert rc == 0 and rel_dev(J, sens["x0"]["du1"]) <= 1e-6


@pytest.mark.parametrize("kind,Hc", [("small", 0), ("small", 5), ("plate", 0)])
def test_shift_matches_oracle_bit_for_bit(kind, Hc):
    """A random iterate placed with set_iterate, shifted by a warm = 2 solve
    that stops before its first step (max_iter 0): the held iterate is the
    oracle's shift of it, exactly (index work)."""
    from oracle.ipm import IPMState
    from oracle.nmpc import shift_state
    from oracle.plate import PlateOCP
    from workloads import plate_workload
    note(f"shifted warm start {kind} Hc {Hc}")
    if kind == "plate":
        w = plate_workload("large", 0, G=8, H=4)
        m = PlateOCP.from_workload(w)
        p = N.Problem(N.plate_structure(8, 4, w.dt, t_hi=w.T_hi, c_lo=w.u_lo, c_hi=w.u_hi))
        p.analyze()
        p.set_parameters(w.T0, setpoint=w.target, u_prev=m.u_prev)
    else:
        w, m, p = _pair("small", 0, Hc)
    rng = np.random.default_rng(7)
    ml = 2 * m.m_c + m.m_d
    st = IPMState(rng.uniform(0.1, 0.9, m.n), *(rng.uniform(0.5, 2.0, ml) for _ in range(3)),
                  rng.uniform(0.1, 1.0, m.n), rng.uniform(0.1, 1.0, m.n))
    p.set_iterate(st.y, st.s, st.omega, st.beta, st.zL, st.zU)
    r = p.solve(warm="shift", options=N.default_options(max_iter=0))
    assert r.iters == 0
    got = p.get_iterate()
    want = shift_state(m, st)
    for key in ("y", "s", "omega", "beta", "zL", "zU"):
        assert np.array_equal(got[key], getattr(want, key)), key


def test_shifted_episode_matches_oracle():
    """Closed loop with shifted warm starts (control horizon 8): every solve
    certified, then both sides tighten their own point and are compared; the
    next solve starts from each side's tightened point shifted by one stage
    (both sides get the same next measurement and last control)."""
    from oracle.nmpc import shift_state
    note("shifted episode, small column Hc 8")
    w, m, p = _pair("small", 1, 8)
    ipm = LiftedIPM(m, IPMOptions(tol=PARITY_TOL))
    x0, u_prev = w.x0.copy(), w.u_prev0.copy()
    st = None
    for i in range(4):
        m.set_parameters(x0=x0, zF=w.zF(i), u_prev=u_prev)
        p.set_parameters(x0, setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(i), u_prev=u_prev)
        if st is None:
            ref = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
        else:
            ref = ipm.solve(shift_state(m, st), ipm.o.mu0_warm)
        r = p.solve(warm="shift" if i > 0 else False, options=N.default_options(tol=PARITY_TOL))
        note(f"solve {i}: iterations gpu {r.iters} oracle {ref.iters}")
        assert r.status == 0 and ref.status == 0 and abs(r.iters - ref.iters) <= 2
        assert r.mu == ipm.o.mu_min and ref.mu == ipm.o.mu_min
        sol = p.solution()
        assert kkt_error(m, sol["y"], sol["lam"], sol["omega_d"], sol["zL"], sol["zU"])["max"] <= 1e-8
        assert p.solve(warm=True, options=N.default_options(fixed_mu=1, tol=TIGHT_TOL, mu0_warm=r.mu,
                                                             max_iter=30)).status == 0
        ref_t = ipm.solve(ref.state, ref.mu, fixed_mu=True, tol=TIGHT_TOL)
        assert ref_t.status == 0
        st = ref_t.state
        lam, nu = ipm.multipliers(st)
        sol = p.solution()
        for key, got, want in (("y", sol["y"], st.y), ("lam", sol["lam"], lam), ("nu", sol["omega_d"], nu),
                               ("zL", sol["zL"], st.zL), ("zU", sol["zU"], st.zU)):
            d = rel_dev(got, want)
            assert d <= 1e-6, (i, key, d)
        u_prev = m.u1(st.y)
        x0 = w.next_measurement(m.x1(st.y), i)


def test_closed_loop_with_plant_model_mismatch():
    """Algorithm 1 against a plant whose relative volatility is 8 % above the
    model's: every solve of the loop converges and is certified for the
    parameters it was given (the measured state, not the prediction), and the
    measured trajectory leaves the matched one."""
    from paper_2606_04725_amd.plant import DistillationPlant
    note("closed loop, plant alpha x 1.08")
    w = distillation_workload("small", 0)
    m = DistillationOCP.from_workload(w)
    traj = {}
    for name, alpha in (("matched", w.alpha), ("mismatched", 1.08 * w.alpha)):
        plant = DistillationPlant(w.N, alpha, w.dt, F=w.F)
        p = N.Problem(N.distillation_structure(w.N, w.H, w.dt, w.alpha, F=w.F, rho=w.rho))
        p.analyze()
        x, up = w.x0.copy(), w.u_prev0.copy()
        xs = []
        for k in range(12):
            p.set_parameters(x, setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(k), u_prev=up)
            r = p.solve(warm=k > 0)
            assert r.status == 0, (name, k, r.status)
            if k % 4 == 0:
                m.set_parameters(x0=x, zF=w.zF(k), u_prev=up)
                sol = p.solution()
                assert kkt_error(m, sol["y"], sol["lam"], sol["omega_d"], sol["zL"], sol["zU"])["max"] <= 1e-8
            u1, _ = p.first_stage()
            x = plant.step(x, u1, zF=float(w.zF(k)[0]))
            up = u1
            xs.append(x.copy())
        traj[name] = np.array(xs)
    assert np.max(np.abs(traj["matched"] - traj["mismatched"])) > 1e-3
