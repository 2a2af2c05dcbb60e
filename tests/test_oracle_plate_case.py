"""Pins for the oracle's heated-plate case study (Section 4.2, Table 2):
complex-step derivatives, the steady state of the discrete heat equation as a
fixed point of the transcription (a sparse direct solve of the independently
assembled Poisson system), the x1 <-> x2 symmetry when both heated edges carry
the same temperature, the trapezoid weights of the tracking region, Table 2's
constants, and a converged solve whose sensitivities match central
differences."""
import numpy as np
import pytest

from oracle.ipm import LiftedIPM
from oracle.kkt import kkt_error
from oracle.plate_case import TABLE2, PlateCaseOCP
from workloads import plate_case_workload

H_CS = 1e-30


def _small(H=3, n=9, loss=50.0):
    m = PlateCaseOCP(H=H, n=n, loss=loss)
    rng = np.random.default_rng(3)
    m.set_parameters(x0=rng.uniform(40.0, 70.0, m.nx), traj=rng.uniform(54.0, 64.0, m.H))
    return m, rng


def _point(m, rng):
    y = rng.uniform(40.0, 70.0, m.n)
    y[m.nx::m.ns] = rng.uniform(0.2, 2.0, m.H)       # q = Q / 1e4
    return y


@pytest.mark.parametrize("n", [9, 21])
def test_complex_step_derivatives(n):
    m, rng = _small(H=2, n=n)
    y = _point(m, rng)
    E = np.eye(m.n)
    g_cs = np.array([m.f(y + 1j * H_CS * E[i]).imag / H_CS for i in range(m.n)])
    assert np.max(np.abs(m.grad(y) - g_cs)) <= 1e-13 * max(1.0, np.max(np.abs(g_cs)))
    J_cs = np.array([m.cons_c(y + 1j * H_CS * E[i]).imag / H_CS for i in range(m.n)]).T
    J = m.jac_c(y).toarray()
    assert np.max(np.abs(J - J_cs)) <= 1e-13 * max(1.0, np.max(np.abs(J_cs)))
    lam = rng.normal(size=m.m_c)
    H_cs = np.array([(m.grad(y + 1j * H_CS * E[i]) + m.jac_c(y + 1j * H_CS * E[i]).T @ lam).imag / H_CS
                     for i in range(m.n)])
    W = m.hess(y, lam, np.zeros(0)).toarray()
    assert np.max(np.abs(W - H_cs)) <= 1e-11 * max(1.0, np.max(np.abs(H_cs)))


def test_steady_state_is_a_fixed_point():
    """The discrete steady state for an input Q (sparse solve of lap_h T = s
    with Q's edges) held at every stage with Q applied makes every row zero."""
    m = PlateCaseOCP(H=4)
    Q = 8300.0
    Ts = m.steady_state(Q)
    m.set_parameters(x0=Ts)
    y = np.tile(np.concatenate([Ts, [Q / m.qs]]), m.H)
    c = m.cons_c(y)
    assert np.max(np.abs(c)) <= 1e-9 * np.max(np.abs(Ts))


def test_symmetry_when_both_heated_edges_match():
    """4.1 Q^(1/3) = Q^(1/2) at Q = 4.1^6: left and bottom edges are equal, so
    the steady state and the transcription commute with x1 <-> x2."""
    m = PlateCaseOCP(H=2)
    Q = 4.1 ** 6
    left, bottom = m.edges(Q)
    assert abs(left - bottom) <= 1e-10 * left
    g = m.g
    Ts = m.steady_state(Q).reshape(g, g)
    assert np.max(np.abs(Ts - Ts.T)) <= 1e-10 * np.max(np.abs(Ts))
    rng = np.random.default_rng(1)
    F = rng.uniform(40, 70, (g, g))
    m.set_parameters(x0=F.reshape(-1), traj=[58.0, 58.0])
    y = np.concatenate([F.reshape(-1), [Q / m.qs], F.T.reshape(-1), [Q / m.qs]])
    m2 = PlateCaseOCP(H=2)
    m2.set_parameters(x0=F.T.reshape(-1), traj=[58.0, 58.0])
    y2 = np.concatenate([F.T.reshape(-1), [Q / m.qs], F.reshape(-1), [Q / m.qs]])
    c1 = m.cons_c(y).reshape(2, g, g)
    c2 = m2.cons_c(y2).reshape(2, g, g)
    assert np.max(np.abs(c1 - np.transpose(c2, (0, 2, 1)))) <= 1e-9
    assert abs(m.f(y) - m2.f(y2)) <= 1e-10 * abs(m.f(y))


def test_tracking_weights_are_the_trapezoid_rule():
    m = PlateCaseOCP(H=1)
    w = m.weights.reshape(m.g, m.g)
    assert abs(w.sum() - 1.0) <= 1e-14                     # area of [-0.5, 0.5]^2
    x1 = np.tile(m.coord, (m.g, 1))
    # trapezoid rule of x1^2 on [-0.5, 0.5] with h = 0.1 (times the x2 length 1)
    want = 0.1 * (0.5 * 0.25 * 2 + 2 * (0.16 + 0.09 + 0.04 + 0.01))
    assert abs((w * x1 * x1).sum() - want) <= 1e-14
    assert np.count_nonzero(w) == 121


def test_table2_constants():
    w = plate_case_workload()
    assert (w.alpha, w.Tb, w.n, w.rho, w.q_loss) == (TABLE2["alpha"], TABLE2["Tb"], TABLE2["n"], TABLE2["rho"],
                                                    TABLE2["q_loss"])
    assert abs(2.0 / (w.n - 1) - TABLE2["L"]) <= 1e-15     # L is the grid spacing
    assert w.loss == 5.0 * w.q_loss                       # the reading of the loss term
    assert list(w.traj(0)[:7]) == [58.0] * 6 + [55.0]
    assert w.traj(19)[0] == 63.0


def _first_solve(loss):
    w = plate_case_workload(loss=loss)
    m = PlateCaseOCP(H=w.H, dt=w.dt, n=w.n, alpha=w.alpha, Tb=w.Tb, loss=w.loss, rho=w.rho, Q_lo=w.Q_lo,
                     q_scale=w.q_scale)
    m.set_parameters(x0=np.full(m.nx, w.T0), traj=w.traj(0), u_prev=[w.Q_prev0 / w.q_scale])
    ipm = LiftedIPM(m)
    res = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
    return m, ipm, res


def test_first_solve_converges_and_the_loss_reading():
    """The first NMPC solve converges (KKT <= 1e-8); with the loss term read
    as 5 q_loss the region's mean temperature comes within a few degrees of
    the 58 setpoint, while the printed 5 q_loss^2 leaves it below 45 at the
    optimum (the rho Q^2 price of the far larger input it would need)."""
    m, ipm, res = _first_solve(50.0)
    assert res.status == 0 and res.iters <= 40
    lam, nu = ipm.multipliers(res.state)
    assert kkt_error(m, res.state.y, lam, nu, res.state.zL, res.state.zU)["max"] <= 1e-8
    T, q = m.split(res.state.y)
    mean = (T @ m.weights) / m.weights.sum()
    assert 53.0 <= mean[0] <= 58.0
    m2, _, res2 = _first_solve(500.0)
    assert res2.status == 0
    T2, _ = m2.split(res2.state.y)
    assert ((T2 @ m2.weights) / m2.weights.sum())[0] < 45.0


def test_sensitivities_match_central_differences():
    from oracle.adjoint import sensitivities
    m, rng = _small(H=3, n=9)
    ipm = LiftedIPM(m)
    res = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
    assert res.status == 0
    mu = res.mu
    st = ipm.solve(res.state, mu, fixed_mu=True, tol=1e-13).state
    sens = sensitivities(ipm, st)
    base = dict(x0=m.x0.copy(), traj=m.traj.copy())
    hstep = 1e-5
    for group, idx in (("x0", 0), ("x0", 24), ("traj", 1)):
        vals = []
        for sgn in (1, -1):
            v = base[group].copy()
            v[idx] += sgn * hstep
            m.set_parameters(**{group: v})
            s2 = ipm.solve(st, mu, fixed_mu=True, tol=1e-13)
            assert s2.status == 0
            vals.append((m.u1(s2.state.y), m.f(s2.state.y)))
        m.set_parameters(**{group: base[group]})
        du_fd = (vals[0][0] - vals[1][0]) / (2 * hstep)
        df_fd = (vals[0][1] - vals[1][1]) / (2 * hstep)
        assert np.max(np.abs(sens[group]["du1"][:, idx] - du_fd)) <= 1e-5 * max(1e-3, np.max(np.abs(du_fd))) + 1e-8
        assert abs(sens[group]["df"][idx] - df_fd) <= 1e-5 * max(1e-3, abs(df_fd)) + 1e-8
