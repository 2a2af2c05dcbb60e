"""Pins for the oracle's solution sensitivities (implicit function theorem on the
lifted barrier KKT conditions, condensed as in eqs. 14 and 17)."""
import numpy as np
import pytest

from oracle.adjoint import sensitivities, vjp
from oracle.distillation import DistillationOCP
from oracle.ipm import LiftedIPM
from oracle.lq import LQOCP, random_lq
from oracle.riccati import riccati_gains
from workloads import distillation_workload


def _solve_cold(m):
    ipm = LiftedIPM(m)
    res = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
    assert res.status == 0
    return ipm, res


@pytest.mark.parametrize("seed", [0, 3])
def test_lq_first_stage_gain(seed):
    """Closed form: u_1* = -K_1 x0 + kff_1, so d u_1*/d x0 = -K_1.  The lifted
    barrier solution approximates the equality-constrained one with a penalty of
    order beta / s on the equalities, so agreement is to a few 1e-7."""
    A, B, Q, R, x0, xs = random_lq(4, 2, 10, seed=seed)
    m = LQOCP(A, B, Q, R, 10, xs=xs)
    m.set_parameters(x0=x0)
    ipm, res = _solve_cold(m)
    sens = sensitivities(ipm, res.state)
    K, _ = riccati_gains(A, B, Q, R, 10, xs)
    assert np.allclose(sens["x0"]["du1"], -K[1], rtol=1e-5, atol=2e-6)


def _fixed_mu_resolve(ipm, m, st, mu, setter, value):
    setter(value)
    res = ipm.solve(st, mu, fixed_mu=True, tol=1e-13)
    assert res.status == 0
    return res.state


def test_distillation_sensitivities_match_central_differences():
    w = distillation_workload("small", 2, N=4, H=4)
    m = DistillationOCP.from_workload(w)
    m.set_parameters(x0=w.x0, zF=w.zF(0), u_prev=w.u_prev0)
    ipm, res = _solve_cold(m)
    mu = res.mu
    # differentiate the barrier problem at its tightly converged solution (the
    # finite differences below perturb that solution)
    st = ipm.solve(res.state, mu, fixed_mu=True, tol=1e-13).state
    base = dict(x0=m.x0.copy(), zF=m.zF.copy(), u_prev=m.u_prev.copy(), setpoint=np.array([m.xD_sp, m.xB_sp]))
    sens = sensitivities(ipm, st)
    h = 1e-6
    checks = [("x0", 0), ("x0", 3), ("x0", m.nx - 1), ("setpoint", 0), ("setpoint", 1), ("zF", 0), ("zF", 2),
              ("u_prev", 0), ("u_prev", 1)]
    for group, idx in checks:
        def setter(v, g=group):
            m.set_parameters(**{g: v})
        vals = []
        for sgn in (+1, -1):
            v = base[group].copy()
            v[idx] += sgn * h
            s2 = _fixed_mu_resolve(ipm, m, st, mu, setter, v)
            vals.append((m.u1(s2.y), m.f(s2.y)))
        setter(base[group])
        du_fd = (vals[0][0] - vals[1][0]) / (2 * h)
        df_fd = (vals[0][1] - vals[1][1]) / (2 * h)
        du = sens[group]["du1"][:, idx]
        df = sens[group]["df"][idx]
        scale = max(1e-3, np.max(np.abs(du_fd)))
        assert np.max(np.abs(du - du_fd)) <= 1e-5 * scale + 1e-7, (group, idx, du, du_fd)
        assert abs(df - df_fd) <= 1e-5 * max(1e-3, abs(df_fd)) + 1e-7, (group, idx, df, df_fd)


def test_setpoint_gradient_envelope_theorem():
    """The optimal value's gradient with respect to a parameter that enters only
    the objective equals the objective's partial derivative at the solution, up
    to the barrier terms: mu sum (ds/dp)/s over the lifted rows is about
    sum lambda dc/dp with c confined to [-gamma, gamma], of order gamma n |lambda|."""
    w = distillation_workload("small", 1)
    m = DistillationOCP.from_workload(w)
    m.set_parameters(x0=w.x0, zF=w.zF(0), u_prev=w.u_prev0)
    ipm, res = _solve_cold(m)
    st = ipm.solve(res.state, res.mu, fixed_mu=True, tol=1e-13).state
    sens = sensitivities(ipm, st)
    X = st.y.reshape(m.H, m.ns)
    partial = np.array([-2.0 * np.sum(X[:, 0] - m.xD_sp), -2.0 * np.sum(X[:, m.nx - 1] - m.xB_sp)])
    assert np.allclose(sens["setpoint"]["df"], partial, rtol=0, atol=1e-5)


def test_vjp_is_seeded_jacobian():
    w = distillation_workload("small", 0, N=3, H=3)
    m = DistillationOCP.from_workload(w)
    m.set_parameters(x0=w.x0, zF=w.zF(0), u_prev=w.u_prev0)
    ipm, res = _solve_cold(m)
    sens = sensitivities(ipm, res.state)
    g = vjp(ipm, res.state, np.array([0.3, -1.1]), 0.7)
    for k in sens:
        assert np.allclose(g[k], np.array([0.3, -1.1]) @ sens[k]["du1"] + 0.7 * sens[k]["df"])


def test_condensed_and_uncondensed_sensitivities_agree():
    """The condensed matrix of eqs. (14)/(17) and the uncondensed system give the
    same sensitivities up to the rounding the condensation carries."""
    from oracle.adjoint import condensed_matrix
    w = distillation_workload("small", 3)
    m = DistillationOCP.from_workload(w)
    m.set_parameters(x0=w.x0, zF=w.zF(0), u_prev=w.u_prev0)
    ipm, res = _solve_cold(m)
    st = res.state
    sens = sensitivities(ipm, st)
    K, Jc, Jd, Qc, Qd = condensed_matrix(ipm, st)
    dc, dd, dgrad, dfp = m.parameter_derivatives(st.y)["x0"]
    dy = np.linalg.solve(K, -dgrad - Jc.T @ (Qc[:, None] * dc) - Jd.T @ (Qd[:, None] * dd))
    assert np.max(np.abs(dy[m.u1_index(), :] - sens["x0"]["du1"])) <= 1e-4 * max(1.0, np.max(np.abs(dy)))


def test_plate_sensitivities_match_central_differences():
    from oracle.plate import PlateOCP
    from workloads import plate_workload
    w = plate_workload("large", 0, G=8, H=3)   # at G = 4 two segments drive the same corner node only
    m = PlateOCP.from_workload(w)
    ipm, res = _solve_cold(m)
    mu = res.mu
    st = ipm.solve(res.state, mu, fixed_mu=True, tol=1e-13).state
    sens = sensitivities(ipm, st)
    base = dict(x0=m.x0.copy(), setpoint=m.target.copy())
    h = 1e-6
    for group, idx in [("x0", 0), ("x0", 5), ("setpoint", 3), ("setpoint", 10)]:
        vals = []
        for sgn in (+1, -1):
            v = base[group].copy()
            v[idx] += sgn * h
            m.set_parameters(**{group: v})
            s2 = ipm.solve(st, mu, fixed_mu=True, tol=1e-13)
            assert s2.status == 0
            vals.append((m.u1(s2.state.y), m.f(s2.state.y)))
        m.set_parameters(**{group: base[group]})
        du_fd = (vals[0][0] - vals[1][0]) / (2 * h)
        df_fd = (vals[0][1] - vals[1][1]) / (2 * h)
        scale = max(1e-3, np.max(np.abs(du_fd)))
        assert np.max(np.abs(sens[group]["du1"][:, idx] - du_fd)) <= 1e-5 * scale + 1e-7, (group, idx)
        assert abs(sens[group]["df"][idx] - df_fd) <= 1e-5 * max(1e-3, abs(df_fd)) + 1e-7, (group, idx)


def test_plate_setpoint_gradient_envelope_theorem():
    """The target field enters only the objective: df*/dT*_p = -2 sum_k (T_kp - T*_p)
    up to the barrier and lifting terms."""
    from oracle.plate import PlateOCP
    from workloads import plate_workload
    w = plate_workload("large", 2, G=8, H=4)
    m = PlateOCP.from_workload(w)
    ipm, res = _solve_cold(m)
    st = ipm.solve(res.state, res.mu, fixed_mu=True, tol=1e-13).state
    sens = sensitivities(ipm, st)
    T = st.y.reshape(m.H, m.ns)[:, :m.nx]
    partial = -2.0 * np.sum(T - m.target[None, :], axis=0)
    assert np.allclose(sens["setpoint"]["df"], partial, rtol=0, atol=1e-5)


def test_toy_sensitivities_match_central_differences():
    """The toy problem of the re-solve listing with an explicit trajectory: d u1
    and d f* with respect to y0 and to the tracked value of two stages, against
    central differences of fixed-mu re-solves (this pins the toy's
    parameter_derivatives, which only the sensitivity solve uses)."""
    from oracle.toy import ToyOCP
    m = ToyOCP()
    m.set_parameters(y0=0.7, traj=np.sin(m.t + 0.4))
    ipm, res = _solve_cold(m)
    mu = res.mu
    st = ipm.solve(res.state, mu, fixed_mu=True, tol=1e-13).state
    sens = sensitivities(ipm, st)
    base = dict(y0=np.array([m.y0]), traj=m.traj.copy())
    h = 1e-6
    for group, idx in (("y0", 0), ("traj", 0), ("traj", 5)):
        def setter(v, g=group):
            m.set_parameters(**{g: (v[0] if g == "y0" else v)})
        vals = []
        for sgn in (+1, -1):
            v = base[group].copy()
            v[idx] += sgn * h
            s2 = _fixed_mu_resolve(ipm, m, st, mu, setter, v)
            vals.append((m.u1(s2.y), m.f(s2.y)))
        setter(base[group])
        du_fd = (vals[0][0] - vals[1][0]) / (2 * h)
        df_fd = (vals[0][1] - vals[1][1]) / (2 * h)
        du = sens[group]["du1"][:, idx]
        df = sens[group]["df"][idx]
        assert np.max(np.abs(du - du_fd)) <= 1e-5 * max(1e-3, np.max(np.abs(du_fd))) + 1e-7, (group, idx, du, du_fd)
        assert abs(df - df_fd) <= 1e-5 * max(1e-3, abs(df_fd)) + 1e-7, (group, idx, df, df_fd)
